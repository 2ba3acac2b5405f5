// Wavefront equality aggregation: the gfx950 analogue of DialSort's Conflict
// Resolution Network (Sec. 6).
//
// The paper's CRN merges concurrent updates of one key into a single additive
// write (Eq. (3): equal keys -> one pair whose count is the sum; Eq. (4): unequal
// keys pass through) and relies only on the conservation of per-key counts
// (Lemma "lem:crn").  On a 64-lane wavefront the same merge is done with
// equality tests and ballots, never with an order comparison (Definition
// "def:ordercomp"):
//   * a candidate key hk (wave-uniform, learnt from earlier slots) gathers every
//     lane holding hk: one lane adds popcount(mask) for all of them;
//   * a discovery step takes the first still-active lane's key as leader and
//     merges every lane holding it the same way; if that group is larger than the
//     candidate's, the leader key becomes the new candidate;
//   * the remaining lanes add 1 each.
// Every key is added exactly once, so the per-key totals are unchanged (the
// additive invariant of Lemma "lem:crn"); which lanes merge only changes the
// number of atomic updates, never the counts.  Uniform keys cost two extra
// ballots per slot; a hot key collapses from up to 64 same-address LDS atomics
// (which serialise) to one.
#pragma once

#include "common.hpp"

namespace ds {

struct WaveAgg {
  uint32_t hk = 0xFFFFFFFFu;  // candidate key (wave-uniform)
};

// Merge one slot (one key per lane, `act` = lane holds a key) and call
// emit(key, count) once per merged group and once per remaining lane.
template <int AGG, typename Emit>
__device__ __forceinline__ void wave_merge(uint32_t x, bool act, WaveAgg& st, Emit& emit) {
  if constexpr (AGG == 0) {
    if (act) emit(x, 1u);
  } else {
    const uint32_t lane = lane_id();
    const bool eq = act && (x == st.hk);
    const uint64_t m = __ballot(eq);
    uint32_t hc = 0;
    if (m) {
      hc = (uint32_t)__popcll(m);
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
      if (lane == leader) emit(st.hk, hc);
      act = act && !eq;
    }
    const uint64_t am = __ballot(act);
    if (am) {
      const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
      const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)ll);
      const bool eq2 = act && (x == lk);
      const uint64_t m2 = __ballot(eq2);
      const uint32_t c = (uint32_t)__popcll(m2);
      if (lane == ll) emit(lk, c);
      act = act && !eq2;
      if (c > hc && c >= 2) st.hk = lk;
    }
    if (act) emit(x, 1u);
  }
}

// Same merge, but every lane also receives its rank among the keys of its group
// in the counter array cnt (the old counter value plus its position within the
// merged group).  Used to place keys into buckets.
template <int AGG>
__device__ __forceinline__ uint32_t wave_rank(uint32_t* cnt, uint32_t b, bool act, WaveAgg& st) {
  if constexpr (AGG == 0) {
    return act ? atomicAdd(&cnt[b], 1u) : 0u;
  } else {
    const uint32_t lane = lane_id();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t r = 0;
    const bool eq = act && (b == st.hk);
    const uint64_t m = __ballot(eq);
    uint32_t hc = 0;
    if (m) {
      hc = (uint32_t)__popcll(m);
      const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
      uint32_t old = 0;
      if (lane == leader) old = atomicAdd(&cnt[st.hk], hc);
      old = (uint32_t)__builtin_amdgcn_readlane((int)old, (int)leader);
      if (eq) r = old + (uint32_t)__popcll(m & below);
      act = act && !eq;
    }
    const uint64_t am = __ballot(act);
    if (am) {
      const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
      const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)b, (int)ll);
      const bool eq2 = act && (b == lk);
      const uint64_t m2 = __ballot(eq2);
      const uint32_t c = (uint32_t)__popcll(m2);
      uint32_t old = 0;
      if (lane == ll) old = atomicAdd(&cnt[lk], c);
      old = (uint32_t)__builtin_amdgcn_readlane((int)old, (int)ll);
      if (eq2) r = old + (uint32_t)__popcll(m2 & below);
      act = act && !eq2;
      if (c > hc && c >= 2) st.hk = lk;
    }
    if (act) r = atomicAdd(&cnt[b], 1u);
    return r;
  }
}

}  // namespace ds
