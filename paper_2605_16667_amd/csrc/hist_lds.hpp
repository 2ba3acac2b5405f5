// Ingestion into LDS-privatized sub-histograms (DialSort Sec. 3.3, Eq. (1)),
// for universes that fit in one workgroup's LDS.
//
// Workgroup g counts the keys of slab [g*per, min((g+1)*per, n)) into an LDS
// histogram of the whole universe and writes it out as row g of a partial
// histogram matrix (or directly as H when there is a single workgroup).  The
// rows are summed by the scan kernel; no global atomics and no zeroing of H are
// needed, and the result does not depend on the order in which workgroups run.
//
//   * LDS32: U <= 32768, one uint32 counter per bin (up to 128 KiB of LDS).
//   * LDS16: 32768 < U <= 65536: two 16-bit counters packed per 32-bit word
//     (128 KiB).  A field that wraps is corrected exactly: every atomic add
//     returns the old word, from which the adding lane sees whether its field
//     crossed a multiple of 65536 (and, for the low field, whether the carry into
//     the high field made that field cross one).  Each crossing is logged as a
//     +-65536 event for its bin; a low-field carry is taken back out of the high
//     field with a second atomic.  The field's final value plus 65536 times its
//     net events is its exact count, in whatever order the adds land.  With at
//     most 2^22 keys per workgroup a workgroup logs at most 256 events (the log
//     holds 512).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "crn_wave.hpp"

namespace ds {

// Load up to 4 keys of group [e0, e0+4) clipped at `end`; returns how many are
// valid (a prefix of v).  Each key is mapped to its index x - lo (mod 2^32),
// the order-isomorphism phi of Sec. 3.4 for a universe that starts at lo.
template <bool ALIGNED>
__device__ __forceinline__ uint32_t load_group(const uint32_t* __restrict__ keys, uint64_t e0, uint64_t end,
                                               uint32_t v[4], uint32_t lo) {
  uint32_t c = 0;
  if (e0 + 4 <= end) {
    if constexpr (ALIGNED) {
      // keys are read once: non-temporal loads keep them from displacing
      // what the next passes read back (the staging, H)
      typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
      const u32x4_t q = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(keys + e0));
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      v[0] = keys[e0]; v[1] = keys[e0 + 1]; v[2] = keys[e0 + 2]; v[3] = keys[e0 + 3];
    }
    c = 4;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = 0;
      if (e0 + i < end) { v[i] = keys[e0 + i]; c = i + 1; }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] -= lo;
  return c;
}

constexpr int LDS16_EVCAP = 512;

// Event log of the packed counters (rare path).
struct Lds16Log {
  uint32_t* evflag;  // one bit per bin: the bin has logged events
  uint32_t* ev;      // bin | (0x80000000 if the event is -65536)
  uint32_t* nev;
  __device__ __forceinline__ void log(uint32_t bin, bool neg) const {
    const uint32_t i = atomicAdd(nev, 1u);
    if (i < LDS16_EVCAP) ev[i] = bin | (neg ? 0x80000000u : 0u);
    atomicOr(&evflag[bin >> 5], 1u << (bin & 31));
  }
};

// The add of count c to bin k (packed word `word`) returned `old`; log the
// crossings it caused.
__device__ __noinline__ void lds16_crossing(uint32_t* words, uint32_t word, uint32_t k, uint32_t c, uint32_t old,
                                            uint32_t* evflag, uint32_t* ev, uint32_t* nev) {
  Lds16Log L;
  L.evflag = evflag;
  L.ev = ev;
  L.nev = nev;
  if ((k & 1u) == 0) {
    L.log(k, false);                                  // the low field crossed
    if ((old >> 16) == 0xFFFFu) L.log(k + 1, false);  // its carry wrapped the high field
    const uint32_t old2 = atomicAdd(&words[word], 0xFFFF0000u);  // take the carry back out
    if ((old2 >> 16) == 0u) L.log(k + 1, true);
  } else {
    L.log(k, false);
  }
}

// LDS state of one ingestion slab: CAP counter words, plus the crossing log of
// the packed layout.
template <int CAP, bool PACKED>
struct HistSmem {
  __align__(16) uint32_t s[CAP];
  uint32_t evflag[PACKED ? 65536 / 32 : 1];
  uint32_t ev[PACKED ? LDS16_EVCAP : 1];
  uint32_t nev;
};

constexpr int SLICE_LOG2 = 8;  // slices of 256 bins (the one-launch sort's scan)
constexpr uint32_t SLICE_BINS = 1u << SLICE_LOG2;

// Count keys [beg, end) into S (NT threads) and write the U exact counts to row.
// The word of bin x is x (uint32 counters) or x >> 1 (packed).  A key > umax
// sets ST_RANGE in *status.  row16 (a slab of fewer than 2^16 keys, row
// 16-byte aligned): the row holds 16-bit counts, bin 2w in the low and bin
// 2w + 1 in the high half of word w; with it, scnt (LDS, zeroed, one word per
// slice of 2^SLICE_LOG2 bins) receives the slab's keys per slice.
template <int NT, bool PACKED, int AGG, bool ALIGNED, int UNR, typename SM>
__device__ __forceinline__ void hist_slab(SM& S, const uint32_t* __restrict__ keys, uint64_t beg, uint64_t end,
                                          uint32_t umax, uint32_t U, uint32_t* __restrict__ row,
                                          uint32_t* status, uint32_t lo = 0, bool row16 = false,
                                          uint32_t* scnt = nullptr) {
  const uint32_t nwords = PACKED ? (U + 1) / 2 : U;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < nwords / 4; i += NT) reinterpret_cast<uint4*>(S.s)[i] = make_uint4(0, 0, 0, 0);
  for (uint32_t i = (nwords & ~3u) + tid; i < nwords; i += NT) S.s[i] = 0;
  if constexpr (PACKED) {
    for (uint32_t i = tid; i < 65536 / 32; i += NT) S.evflag[i] = 0;
    if (tid == 0) S.nev = 0;
  }
  __syncthreads();

  bool bad = false;
  WaveAgg st;
  // AGG 6: the wave's candidate key hk is counted in registers -- each lane
  // adds its matches to acc, no LDS atomic -- and the sum goes to LDS in one
  // add when the candidate changes, when the slab ends and (packed counters)
  // every HOT_FLUSH_ITERS iterations, so that a flush adds less than 2^16
  // (at most 33 iterations of 64 * 4 * UNR keys) and crosses a field boundary
  // at most once.
  constexpr uint32_t HOT_FLUSH_ITERS = (1u << 15) / (WAVE * 4 * UNR);
  uint32_t hk = 0xFFFFFFFFu;  // wave-uniform; no index <= umax < 2^32 - 1 equals it
  uint32_t acc = 0, since = 0;
  auto flush = [&]() {
    const uint32_t c = __builtin_amdgcn_readfirstlane(wave_sum(acc));
    acc = 0;
    since = 0;
    if (c == 0) return;
    if (lane_id() == 0) {
      if constexpr (!PACKED) {
        atomicAdd(&S.s[hk], c);
      } else {
        const uint32_t old = atomicAdd(&S.s[hk >> 1], c << ((hk & 1u) << 4));
        if (__builtin_amdgcn_ubfe(old, (hk & 1u) << 4, 16) + c >= 0x10000u)
          lds16_crossing(S.s, hk >> 1, hk, c, old, S.evflag, S.ev, &S.nev);
      }
    }
  };
  // One slot of AGG 6 / 8: cin is the lane's count for its key in this slot
  // (1, or with AGG 8 its run's length, 0 for an invalid or merged key);
  // returns what the lane adds to its key's bin, after counting a match of
  // the candidate in registers.  The
  // first slot of every iteration (probe) also looks for a group of
  // AGG_HOT_MIN or more lanes on one key other than the candidate; a group
  // larger than the candidate's in that slot takes its place, so the
  // candidate settles on the key most lanes share.
  auto slot_count6 = [&](uint32_t x, uint32_t cin, bool probe) -> uint32_t {
    const bool ok = cin != 0;
    const bool eq = ok && x == hk;
    acc += eq ? cin : 0u;
    bool act = ok && !eq;
    if (probe) {
      const uint64_t am = __ballot(act);
      if (am) {
        const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
        const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)ll);
        const bool eq2 = act && x == lk;
        const uint32_t c2 = (uint32_t)__popcll(__ballot(eq2));
        if (c2 >= AGG_HOT_MIN && c2 > (uint32_t)__popcll(__ballot(eq))) {
          flush();
          hk = lk;
          acc = eq2 ? cin : 0u;
          act = act && !eq2;
        }
      }
    }
    return act ? cin : 0u;
  };
  // AGG 8 adds the lane-local merge (a3): the 4 keys a lane loads together
  // are consecutive in memory, and a run of equal ones among them is counted
  // once, by its first key carrying the run's length (equality tests only);
  // the others carry 0.  run[i] is that count; ok[i] marks valid keys.
  auto lane_runs = [&](const uint32_t (&x)[4], const bool (&ok)[4], uint32_t (&run)[4]) {
    bool eqn[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) eqn[i] = ok[i] && ok[i + 1] && x[i] == x[i + 1];
    uint32_t r = ok[3] ? 1u : 0u;
    run[3] = r;
#pragma unroll
    for (int i = 2; i >= 0; --i) {
      r = ok[i] ? (eqn[i] ? r + 1 : 1u) : 0u;
      run[i] = r;
    }
#pragma unroll
    for (int i = 1; i < 4; ++i) run[i] = eqn[i - 1] ? 0u : run[i];
  };
  // uniform trip count across the workgroup: every lane takes part in the ballots
  for (uint64_t g0 = beg; g0 < end; g0 += (uint64_t)NT * 4 * UNR) {
    if constexpr (AGG >= 6 && PACKED) {
      if (++since > HOT_FLUSH_ITERS) flush();
    }
    uint32_t v[UNR][4];
    uint32_t nv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) nv[u] = load_group<ALIGNED>(keys, g0 + ((uint64_t)u * NT + tid) * 4, end, v[u], lo);
    uint32_t cc[UNR][4];
    uint32_t old[UNR][4];
    // a step whose groups are all whole and whose keys are all in range (every
    // step but the last and those of a faulty input) needs no per-key masks
    uint32_t vmax = 0;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) vmax = vmax > v[u][i] ? vmax : v[u][i];
    const bool clean = g0 + (uint64_t)NT * 4 * UNR <= end && !__any(vmax > umax);
    if (clean) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        uint32_t run[4] = {1u, 1u, 1u, 1u};
        if constexpr (AGG == 8) {
          const bool all[4] = {true, true, true, true};
          lane_runs(v[u], all, run);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          uint32_t c;
          if constexpr (AGG >= 6) {
            c = slot_count6(v[u][i], run[i], u == 0 && i == 0);
          } else {
            WaveGroups g;
            c = wave_merge_count<AGG>(v[u][i], true, st, g);
          }
          cc[u][i] = c;
          old[u][i] = 0;
          if constexpr (!PACKED) {
            if (c) atomicAdd(&S.s[v[u][i]], c);
          } else {
            if (c) old[u][i] = atomicAdd(&S.s[v[u][i] >> 1], c << ((v[u][i] & 1u) << 4));
          }
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        bool oks[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool valid = (uint32_t)i < nv[u];
          oks[i] = valid && v[u][i] <= umax;
          bad |= valid && !oks[i];
        }
        uint32_t run[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) run[i] = oks[i] ? 1u : 0u;
        if constexpr (AGG == 8) lane_runs(v[u], oks, run);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool ok = oks[i];
          uint32_t c;
          if constexpr (AGG >= 6) {
            c = slot_count6(v[u][i], run[i], u == 0 && i == 0);
          } else {
            WaveGroups g;
            c = wave_merge_count<AGG>(v[u][i], ok, st, g);
          }
          cc[u][i] = c;
          old[u][i] = 0;
          if constexpr (!PACKED) {
            if (c) atomicAdd(&S.s[v[u][i]], c);
          } else {
            if (c) old[u][i] = atomicAdd(&S.s[v[u][i] >> 1], c << ((v[u][i] & 1u) << 4));
          }
        }
      }
    }
    if constexpr (PACKED) {
      // crossing checks after every add of the iteration has been issued: a
      // field crossed iff its old value plus the add exceeds 0xFFFF, so one OR
      // over the iteration tells whether any did
      uint32_t anyx = 0;
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) anyx |= __builtin_amdgcn_ubfe(old[u][i], (v[u][i] & 1u) << 4, 16) + cc[u][i];
      }
      if (anyx > 0xFFFFu) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint32_t c = cc[u][i], k = v[u][i];
            const uint32_t field = __builtin_amdgcn_ubfe(old[u][i], (k & 1u) << 4, 16);
            if (c && field + c >= 0x10000u) lds16_crossing(S.s, k >> 1, k, c, old[u][i], S.evflag, S.ev, &S.nev);
          }
        }
      }
    }
  }
  if constexpr (AGG >= 6) flush();
  if (__syncthreads_or(bad) && tid == 0) atomicOr(status, ST_RANGE);

  if (row16) {
    // no count reaches 2^16, so no packed field wrapped and the packed words
    // are the row as they stand; uint32 counters are paired
    if constexpr (PACKED) {
      if (tid == 0 && S.nev) atomicOr(status, ST_INT_EVLOG);  // cannot happen below 2^16 keys
    }
    auto word = [&](uint32_t w) -> uint32_t {
      if constexpr (PACKED) return S.s[w];
      else return S.s[2 * w] | ((2 * w + 1 < U ? S.s[2 * w + 1] : 0u) << 16);
    };
    auto fsum = [](uint32_t x) { return (x & 0xFFFFu) + (x >> 16); };
    const uint32_t nw = (U + 1) / 2, nq = nw / 4;
    uint4* row4 = reinterpret_cast<uint4*>(row);
    // quad q holds bins 8q .. 8q + 7, so the 32 quads of a half-wave (one
    // iteration) are one slice: its sum goes to scnt with one add
    for (uint32_t q0 = 0; q0 < nq; q0 += NT) {  // uniform trip count: every lane takes part in the sums
      const uint32_t q = q0 + tid;
      uint32_t c = 0;
      if (q < nq) {
        uint4 x;
        if constexpr (PACKED) x = *reinterpret_cast<const uint4*>(&S.s[4 * q]);
        else x = make_uint4(word(4 * q), word(4 * q + 1), word(4 * q + 2), word(4 * q + 3));
        row4[q] = x;
        c = fsum(x.x) + fsum(x.y) + fsum(x.z) + fsum(x.w);
      }
      if (scnt) {
        c = half_wave_sum(c);
        if ((lane_id() & 31u) == 31u && c) atomicAdd(&scnt[q >> (SLICE_LOG2 - 3)], c);
      }
    }
    for (uint32_t w = 4 * nq + tid; w < nw; w += NT) {
      const uint32_t x = word(w);
      row[w] = x;
      if (scnt && x) atomicAdd(&scnt[(2 * w) >> SLICE_LOG2], fsum(x));
    }
    return;
  }
  if constexpr (!PACKED) {
    for (uint32_t i = tid; i < U; i += NT) row[i] = S.s[i];
  } else {
    const uint32_t ne = S.nev < LDS16_EVCAP ? S.nev : LDS16_EVCAP;
    const bool r8 = (reinterpret_cast<uintptr_t>(row) & 7u) == 0;  // a pair of bins per 8-byte store
    if (tid == 0 && S.nev > LDS16_EVCAP) atomicOr(status, ST_INT_EVLOG);  // cannot happen within the key bound
    for (uint32_t w = tid; w < nwords; w += NT) {
      const uint32_t word = S.s[w];
      uint64_t cnt[2] = {word & 0xFFFFu, word >> 16};
      if ((S.evflag[(2 * w) >> 5] >> ((2 * w) & 31)) & 3u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t bin = 2 * w + h;
          if (S.evflag[bin >> 5] & (1u << (bin & 31))) {
            for (uint32_t e = 0; e < ne; ++e) {
              const uint32_t x = S.ev[e];
              if ((x & 0x7FFFFFFFu) == bin) cnt[h] += (x & 0x80000000u) ? (uint64_t)-65536ll : 65536ull;
            }
          }
        }
      }
      if (r8 && 2 * w + 1 < U) {
        *reinterpret_cast<uint2*>(row + 2 * w) = make_uint2((uint32_t)cnt[0], (uint32_t)cnt[1]);
      } else {
        row[2 * w] = (uint32_t)cnt[0];
        if (2 * w + 1 < U) row[2 * w + 1] = (uint32_t)cnt[1];
      }
    }
  }
}

// NT threads; CAP = LDS words; PACKED selects the 16-bit layout.
// rows: G rows of `row_stride` uint32 each (row g at rows + g*row_stride).
// init (partial rows in the workspace, row_stride > U): the launch also does
// what a clearing launch before it would -- block 0 zeroes the control block,
// all blocks zero the nclear look-back words of the scan that follows
// (clear_tiles) -- and each block reports a key past U in its own row, word U
// (zeroed by the block first), which the scan folds into the status.  No block
// touches the control block's status then, so clearing it cannot race with a
// report.  row16: per < 2^16 and the rows are 16-byte aligned (16-bit rows).
template <int NT, int CAP, bool PACKED, int AGG, bool ALIGNED, int UNR>
__global__ __launch_bounds__(NT) void k_hist_lds(const uint32_t* __restrict__ keys, uint64_t n, uint64_t per,
                                                 uint32_t umax, uint32_t U, uint32_t* __restrict__ rows,
                                                 uint64_t row_stride, Ctl* ctl, uint32_t lo, uint32_t init,
                                                 uint64_t* __restrict__ clear_tiles, uint64_t nclear, uint32_t row16) {
  __shared__ HistSmem<CAP, PACKED> S;
  const uint64_t beg = (uint64_t)blockIdx.x * per;
  const uint64_t end = beg + per < n ? beg + per : n;
  uint32_t* row = rows + (uint64_t)blockIdx.x * row_stride;
  uint32_t* status = &ctl->status;
  if (init) {
    if (blockIdx.x == 0 && threadIdx.x < sizeof(Ctl) / 4) reinterpret_cast<uint32_t*>(ctl)[threadIdx.x] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x; i < nclear; i += (uint64_t)gridDim.x * NT)
      clear_tiles[i] = 0;
    status = row + U;
    if (threadIdx.x == 0) *status = 0;  // the same thread reports into it, after barriers
  }
  hist_slab<NT, PACKED, AGG, ALIGNED, UNR>(S, keys, beg, end, umax, U, row, status, lo, row16 != 0);
}

// Direct global atomics into a zeroed H, after the same wave merge.  Used when
// n is small next to U, or U is too large for the partitioned path.
template <int NT, int AGG, bool ALIGNED>
__global__ __launch_bounds__(NT) void k_hist_global(const uint32_t* __restrict__ keys, uint64_t n, uint32_t umax,
                                                    uint32_t* __restrict__ H, Ctl* ctl, uint32_t lo) {
  bool bad = false;
  WaveAgg st;
  const uint64_t stride = (uint64_t)gridDim.x * NT * 4;
  for (uint64_t g0 = (uint64_t)blockIdx.x * NT * 4; g0 < n; g0 += stride) {
    uint32_t v[4];
    const uint32_t c = load_group<ALIGNED>(keys, g0 + (uint64_t)threadIdx.x * 4, n, v, lo);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool valid = (uint32_t)i < c;
      const bool ok = valid && v[i] <= umax;
      bad |= valid && !ok;
      wave_count<AGG>(H, v[i], ok, st);
    }
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) set_status(ctl, ST_RANGE);
}

}  // namespace ds
