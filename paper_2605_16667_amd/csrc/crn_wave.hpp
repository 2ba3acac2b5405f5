// Wavefront equality aggregation: the gfx950 analogue of DialSort's Conflict
// Resolution Network (Sec. 6).
//
// The paper's CRN merges concurrent updates of one key into a single additive
// write (Eq. (3): equal keys -> one pair whose count is the sum; Eq. (4): unequal
// keys pass through) and relies only on the conservation of per-key counts
// (Lemma "lem:crn").  On a 64-lane wavefront the same merge is done with
// equality tests and ballots, never with an order comparison (Definition
// "def:ordercomp").  For one slot (one key per lane):
//   * candidate: every lane holding the wave's candidate key hk (wave-uniform,
//     learnt from earlier slots) joins one group;
//   * discovery: the first still-active lane's key leads a second group; when
//     that group is larger than the candidate's, its key becomes the candidate;
//   * each group's lowest lane carries the group size, the other members carry
//     0; every remaining lane carries 1.
// Afterwards every lane issues at most one atomic add (of its carried count),
// so a slot costs one atomic instruction whatever the merge found.  Every key is
// counted exactly once, so per-key totals are unchanged (the additive invariant
// of Lemma "lem:crn"); the merge only changes how many atomic updates reach a
// bin, which is what serialises same-address LDS atomics under skew.
//
// AGG selects the policy: 0 = no merge; 1 = candidate + discovery on every slot;
// 2 = the candidate test on every slot, discovery on every 8th slot and after a
// slot whose discovery found a group; 3 = hot/cold: in cold mode slots go
// straight to their atomics and only every 16th slot runs a discovery; a
// discovered group of at least 4 lanes switches the wave to hot mode, where the
// candidate test runs on every slot until 16 slots in a row find no group of 4.
// Uniform keys then cost about one scalar test per slot, while a hot key still
// collapses to one atomic per slot.
#pragma once

#include "common.hpp"

namespace ds {

struct WaveAgg {
  uint32_t hk = 0xFFFFFFFFu;  // candidate key (wave-uniform)
  uint32_t slot = 15;         // slots seen (wave-uniform); AGG 3 probes on the first slot
  bool probe = true;          // run discovery on this slot (wave-uniform)
  uint32_t hot = 0;           // AGG 3: slots left in hot mode (wave-uniform)
};

constexpr uint32_t AGG_HOT_TTL = 16;
constexpr uint32_t AGG_HOT_MIN = 4;

// Group bookkeeping of one slot, for ranking.
struct WaveGroups {
  uint64_t m1 = 0, m2 = 0;  // member masks of the candidate and discovery groups
  uint32_t l1 = 0, l2 = 0;  // their lowest lanes
};

template <int AGG>
__device__ __forceinline__ uint32_t wave_merge_count(uint32_t x, bool act, WaveAgg& st, WaveGroups& g) {
  if constexpr (AGG == 0) {
    return act ? 1u : 0u;
  } else if constexpr (AGG == 3) {
    const uint32_t lane = lane_id();
    uint32_t c = act ? 1u : 0u;
    uint32_t hc = 0;
    if (st.hot) {
      const bool eq = act && (x == st.hk);
      g.m1 = __ballot(eq);
      hc = (uint32_t)__popcll(g.m1);
      if (g.m1) {
        g.l1 = (uint32_t)__ffsll((unsigned long long)g.m1) - 1;
        if (eq) c = (lane == g.l1) ? hc : 0u;
        act = act && !eq;
      }
      st.hot = hc >= AGG_HOT_MIN ? AGG_HOT_TTL : st.hot - 1;
    }
    if (((++st.slot) & 15u) == 0u) {
      const uint64_t am = __ballot(act);
      if (am) {
        const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)ll);
        const bool eq2 = act && (x == lk);
        g.m2 = __ballot(eq2);
        g.l2 = ll;
        const uint32_t cc = (uint32_t)__popcll(g.m2);
        if (eq2) c = (lane == ll) ? cc : 0u;
        if (cc >= AGG_HOT_MIN && cc > hc) {
          st.hk = lk;
          st.hot = AGG_HOT_TTL;
        }
      }
    }
    return c;
  } else {
    const uint32_t lane = lane_id();
    uint32_t c = act ? 1u : 0u;
    uint32_t hc = 0;
    const bool eq = act && (x == st.hk);
    g.m1 = __ballot(eq);
    if (g.m1) {
      hc = (uint32_t)__popcll(g.m1);
      g.l1 = (uint32_t)__ffsll((unsigned long long)g.m1) - 1;
      if (eq) c = (lane == g.l1) ? hc : 0u;
      act = act && !eq;
    }
    bool found = false;
    if (AGG == 1 || st.probe) {
      const uint64_t am = __ballot(act);
      if (am) {
        const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)ll);
        const bool eq2 = act && (x == lk);
        g.m2 = __ballot(eq2);
        g.l2 = ll;
        const uint32_t cc = (uint32_t)__popcll(g.m2);
        if (eq2) c = (lane == ll) ? cc : 0u;
        found = cc >= 2;
        if (cc > hc && cc >= 2) st.hk = lk;
      }
    }
    if constexpr (AGG == 2) {
      ++st.slot;
      st.probe = found || ((st.slot & 7u) == 0u);
    }
    return c;
  }
}

// Merge, then count into cnt: returns nothing, one atomic per contributing lane.
template <int AGG>
__device__ __forceinline__ void wave_count(uint32_t* cnt, uint32_t x, bool act, WaveAgg& st) {
  WaveGroups g;
  const uint32_t c = wave_merge_count<AGG>(x, act, st, g);
  if (c) atomicAdd(&cnt[x], c);
}

// Merge, then reserve places in counter cnt[b]: every lane that holds a key gets
// its rank (the counter's old value plus its position in its group).
template <int AGG>
__device__ __forceinline__ uint32_t wave_rank(uint32_t* cnt, uint32_t b, bool act, WaveAgg& st) {
  WaveGroups g;
  const uint32_t c = wave_merge_count<AGG>(b, act, st, g);
  uint32_t old = 0;
  if (c) old = atomicAdd(&cnt[b], c);
  if constexpr (AGG == 0) {
    return old;
  } else {
    const uint32_t lane = lane_id();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t r = old;
    if (g.m1) {
      const uint32_t o1 = (uint32_t)__builtin_amdgcn_readlane((int)old, (int)g.l1);
      if ((g.m1 >> lane) & 1ull) r = o1 + (uint32_t)__popcll(g.m1 & below);
    }
    if (g.m2) {
      const uint32_t o2 = (uint32_t)__builtin_amdgcn_readlane((int)old, (int)g.l2);
      if ((g.m2 >> lane) & 1ull) r = o2 + (uint32_t)__popcll(g.m2 & below);
    }
    return r;
  }
}

// Ranking in two phases, so that the atomics of many slots are in flight at
// once: wave_rank_issue() merges one slot and issues its atomic, returning the
// old counter value (valid for lanes that added) plus, for members of a merged
// group, the lane that added for them and their position in the group;
// wave_rank_finish() turns that into the lane's rank once the atomics are back.
struct RankTicket {
  uint32_t old;   // counter value returned to this lane (if it added)
  uint32_t src;   // lane whose old value applies to this lane
  uint32_t off;   // position within the merged group
  bool grouped;   // wave-uniform: this slot merged a group
};

template <int AGG>
__device__ __forceinline__ RankTicket wave_rank_issue(uint32_t* cnt, uint32_t b, bool act, WaveAgg& st) {
  WaveGroups g;
  const uint32_t c = wave_merge_count<AGG>(b, act, st, g);
  RankTicket tk;
  tk.old = 0;
  if (c) tk.old = atomicAdd(&cnt[b], c);
  const uint32_t lane = lane_id();
  tk.src = lane;
  tk.off = 0;
  tk.grouped = (g.m1 | g.m2) != 0;
  if (tk.grouped) {
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if ((g.m1 >> lane) & 1ull) { tk.src = g.l1; tk.off = (uint32_t)__popcll(g.m1 & below); }
    if ((g.m2 >> lane) & 1ull) { tk.src = g.l2; tk.off = (uint32_t)__popcll(g.m2 & below); }
  }
  return tk;
}

__device__ __forceinline__ uint32_t wave_rank_finish(const RankTicket& tk) {
  if (!tk.grouped) return tk.old;
  return (uint32_t)__shfl((int)tk.old, (int)tk.src, WAVE) + tk.off;
}

}  // namespace ds
