// U-range-partitioned ingestion and projection for universes larger than one
// workgroup's LDS.
//
// The paper leaves large universes to a "hierarchical" scheme it lists as future
// work (Sec. 16 and Sec. 17); this two-pass design is ours.  The universe is cut
// into B buckets of W = 2^16 consecutive keys (bucket of x = x >> 16).
//
// Pass 1 (k_partition): workgroup t takes tile t of TK = 8192 keys, counts them
// per bucket, scans the counts and places every key at a cursor of its bucket
// (LDS atomics, after the wavefront equality merge).  It writes the tile's keys
// grouped by bucket as uint16 bucket-relative keys (x & 0xFFFF) into its own
// slice of the staging buffer, plus the tile's B+1 segment starts seg[t][0..B]
// (seg[t][B] = number of valid keys of the tile).  Staging stays tile-major, so
// every write is a coalesced 16-byte store and no global counter is needed.
//
// Pass 2 (k_bucket): workgroup b first sums seg[t][b] over all tiles -- the number
// of keys in buckets before b, i.e. where bucket b's sorted run starts -- and its
// own segment sizes.  It then gathers segment b of every tile (each lane owns
// whole segments, loads them as aligned 16-byte quads and prefetches the next
// step while counting the current one) into a packed LDS histogram of W bins
// (two 16-bit fields per word, with the exact crossing accounting of the LDS16
// ingestion path), and stores bins [b*W, min((b+1)*W, U)) of H: written once,
// with plain stores, no zeroing and no global atomics.  For the projection
// (Eq. (2)) each thread takes 64 consecutive bins; a block scan of their sums
// gives every thread where its stretch of the bucket's run starts, and it
// appends the fill items (tile-by-chunk pieces of the output, see scan_fill.hpp)
// that start there.  k_fill then writes the whole output with many workgroups
// per CU and fully coalesced stores, whatever the skew.  A bucket with more than
// 2^22 keys is counted in two halves with 32-bit LDS counters (reading its
// segments twice), which keeps the packed path's event log bounded.  Buckets are
// mapped so that each XCD (blockIdx mod 8) takes a contiguous range of them,
// which keeps neighbouring segments and segment-table lines in one L2.
#pragma once

#include "common.hpp"
#include "crn_wave.hpp"
#include "hist_lds.hpp"
#include "scan_fill.hpp"

namespace ds {

constexpr int PART_LOG2W = 16;   // bucket width of the single-array path
constexpr uint32_t PART_W = 1u << PART_LOG2W;
constexpr int PART_TK = 8192;    // keys per pass-1 tile (segment starts fit in uint16)
constexpr int PART_NT = 1024;    // pass-2 workgroup
constexpr int P1_NT = 512;       // pass-1 workgroup (two per CU)
constexpr uint32_t PART_BMAX = 8192;
constexpr uint64_t PART_UMAX = (uint64_t)PART_W * PART_BMAX;  // 2^29

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
template <int NT, int BMAXT, int TK>
struct PartSmem {
  uint32_t cnt[BMAXT + 1];
  __align__(16) uint16_t stage[TK];
  uint32_t scan_tmp[NT / WAVE + 1];
};

// Tile `tile` of TK keys (NT threads; TK <= 65536 so segment starts fit in uint16).  seg: T rows of `bstride` uint16
// (bstride >= B + 1, multiple of 8).  Invalid keys are parked as 0xFFFFFFFF
// (U <= 2^29 here, so no valid key has that value).  Bucket of x: x >> LOG2W.
template <int NT, int BMAXT, int AGG, bool ALIGNED, int LOG2W, int TK>
__device__ __forceinline__ void partition_tile(PartSmem<NT, BMAXT, TK>& S, const uint32_t* __restrict__ keys, uint64_t n,
                                               uint32_t umax, uint32_t B, uint16_t* __restrict__ staging,
                                               uint16_t* __restrict__ seg, uint32_t bstride, uint32_t* status,
                                               uint32_t tile) {
  constexpr int GPT = TK / 4 / NT;  // key groups of 4 per thread
  static_assert(GPT >= 1, "a tile gives every thread at least one group");
  constexpr uint32_t WM = (1u << LOG2W) - 1;
  const uint32_t tid = threadIdx.x;
  const uint64_t tb = (uint64_t)tile * TK;
  const uint64_t te = tb + TK < n ? tb + TK : n;

  for (uint32_t i = tid; i <= B; i += NT) S.cnt[i] = 0;

  uint32_t v[GPT][4];
  bool bad = false;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const uint32_t c = load_group<ALIGNED>(keys, tb + ((uint64_t)u * NT + tid) * 4, te, v[u]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool valid = (uint32_t)i < c;
      const bool ok = valid && v[u][i] <= umax;
      bad |= valid && !ok;
      if (!ok) v[u][i] = 0xFFFFFFFFu;
    }
  }
  // Equality merging pays only where many lanes share a bucket: a tile takes
  // it when some wave finds 8 or more of its first 64 keys (one per lane) in
  // the bucket of its lowest lane's key.  Either way every count is exact.
  bool crowd = false;
  if constexpr (AGG != 0) {
    const uint32_t x0 = v[0][0];
    const uint32_t bk = x0 != 0xFFFFFFFFu ? x0 >> LOG2W : 0xFFFFFFFFu;
    const uint32_t lead = __builtin_amdgcn_readfirstlane(bk);
    crowd = lead != 0xFFFFFFFFu && __popcll(__ballot(bk == lead)) >= 8;
  }
  const bool merge = __syncthreads_or(crowd);
  WaveAgg st;
  if (merge) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool ok = v[u][i] != 0xFFFFFFFFu;
        wave_count<AGG>(S.cnt, ok ? (v[u][i] >> LOG2W) : 0u, ok, st);
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool ok = v[u][i] != 0xFFFFFFFFu;
        wave_count<0>(S.cnt, ok ? (v[u][i] >> LOG2W) : 0u, ok, st);
      }
    }
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(status, ST_RANGE);

  // exclusive scan of the B+1 counters (counter B stays 0, so the total is the
  // number of valid keys); each thread owns a run of CPT counters
  constexpr int CPT = (BMAXT + 1 + NT - 1) / NT;
  uint32_t loc[CPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    loc[j] = i <= B ? S.cnt[i] : 0;
    sum += loc[j];
  }
  uint32_t total;
  uint32_t pre = block_exclusive_sum<NT>(sum, S.scan_tmp, &total);
  uint16_t* srow = seg + (uint64_t)tile * bstride;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    if (i <= B) { S.cnt[i] = pre; srow[i] = (uint16_t)pre; }
    pre += loc[j];
  }
  __syncthreads();

  // place the relative keys at cursors taken from the bucket starts, RG groups
  // of 4 keys at a time: that round's cursor atomics first, then its stores
  constexpr int RG = GPT < 4 ? GPT : 4;
  if (merge) {
    WaveAgg st2;
#pragma unroll
    for (int u0 = 0; u0 < GPT; u0 += RG) {
      RankTicket tk[RG][4];
#pragma unroll
      for (int u = 0; u < RG; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t x = v[u0 + u][i];
          const bool ok = x != 0xFFFFFFFFu;
          tk[u][i] = wave_rank_issue<AGG>(S.cnt, ok ? (x >> LOG2W) : 0u, ok, st2);
        }
      }
#pragma unroll
      for (int u = 0; u < RG; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t x = v[u0 + u][i];
          const uint32_t pos = wave_rank_finish(tk[u][i]);
          if (x != 0xFFFFFFFFu) S.stage[pos] = (uint16_t)(x & WM);
        }
      }
    }
  } else {
    // one returning atomic per key, RG groups in flight
#pragma unroll
    for (int u0 = 0; u0 < GPT; u0 += RG) {
      uint32_t pos[RG][4];
#pragma unroll
      for (int u = 0; u < RG; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t x = v[u0 + u][i];
          pos[u][i] = 0;
          if (x != 0xFFFFFFFFu) pos[u][i] = atomicAdd(&S.cnt[x >> LOG2W], 1u);
        }
      }
#pragma unroll
      for (int u = 0; u < RG; ++u) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t x = v[u0 + u][i];
          if (x != 0xFFFFFFFFu) S.stage[pos[u][i]] = (uint16_t)(x & WM);
        }
      }
    }
  }
  __syncthreads();

  // tile slice of staging: the valid keys, bucket-major, as 16-byte stores
  uint16_t* dst = staging + tb;
  const uint32_t n8 = (total + 7) / 8;
  for (uint32_t i = tid; i < n8; i += NT)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(S.stage)[i];
  __syncthreads();  // S is reused by the caller's next tile
}

template <int BMAXT, int AGG, bool ALIGNED>
__global__ __launch_bounds__(P1_NT) void k_partition(const uint32_t* __restrict__ keys, uint64_t n,
                                                     uint32_t umax, uint32_t B,
                                                     uint16_t* __restrict__ staging,
                                                     uint16_t* __restrict__ seg, uint32_t bstride, Ctl* ctl) {
  __shared__ PartSmem<P1_NT, BMAXT, PART_TK> S;
  partition_tile<P1_NT, BMAXT, AGG, ALIGNED, PART_LOG2W, PART_TK>(S, keys, n, umax, B, staging, seg, bstride, &ctl->status,
                                                         blockIdx.x);
}

// ---------------------------------------------------------------------------
// Pass 2 helpers
// ---------------------------------------------------------------------------

constexpr int BK_SQ = 4;            // 16-byte quads (8 keys each) per lane per gather chunk
constexpr uint32_t BK_LRCAP = 256;  // long-run list entries

// LDS state of a bucket (or of a row sum): counters of one bucket of W = 2^LOG2W
// bins -- packed 16-bit pairs when LOG2W == 16, else one uint32 per bin -- the
// crossing log used by the packed LDS ingestion (hist_slab), the long-run list
// of the item emitter and block-reduction space.
template <int NT, int LOG2W>
struct BinSmem {
  static constexpr bool PACKED = LOG2W == 16;
  static constexpr uint32_t WORDS = PACKED ? (1u << 15) : (1u << LOG2W);
  uint32_t s[WORDS];
  uint32_t evflag[PACKED ? 65536 / 32 : 1];
  uint32_t ev[PACKED ? LDS16_EVCAP : 1];
  uint32_t nev;
  uint32_t lr_k[BK_LRCAP], lr_n[BK_LRCAP], lr_l[BK_LRCAP], lr_i[BK_LRCAP];
  uint64_t lr_o[BK_LRCAP], lr_c[BK_LRCAP], lr_e[BK_LRCAP];
  uint64_t red[NT / WAVE + 1];
  uint32_t n, item0;
};

enum GatherMode { GM_PACKED, GM_HALF, GM_DIRECT };

// Gather the segments of bucket b and count their relative keys.  GM_PACKED:
// into the packed 16-bit fields (W = 2^16), with no check for a field passing
// 0xFFFF -- the caller detects any wrap afterwards from the sum of the fields.
// GM_HALF: 32-bit counters for the keys whose relative value lies in half
// `half` (x >> 15 == half, W = 2^16).  GM_DIRECT: 32-bit counters for all keys
// (W <= 2^15).
// Tiles go to the waves in groups of 64, one tile per lane: group g to wave
// g mod NW, or, with fewer groups than waves, NW / G waves to each group,
// which split its quads between them.  A lane holds its tile's segment
// [s, e) of tile-local key indices and the wave walks the segments of the
// group in chunks of BK_SQ 16-byte quads (8 keys each) per lane, all lanes in
// step, up to the group's longest segment.  Every lane issues every load of a
// chunk -- past the end of its segment it reads the segment's last quad again,
// and without a segment quad 0 -- so the loads have no branches around them
// and stay in flight together; masks keep keys outside [s, e) out of the count.
// The bounds of a wave's next group are loaded before its current group is
// counted.
template <int NT, int LOG2W, int AGG, GatherMode GM, int TK>
__device__ __forceinline__ void bucket_gather(BinSmem<NT, LOG2W>& S, const uint16_t* __restrict__ staging,
                                              const uint16_t* __restrict__ seg, uint32_t bstride, uint32_t T,
                                              uint32_t b, uint32_t half) {
  static_assert(TK % 8 == 0 && TK <= 32768, "tile-local key indices and quad offsets fit 16 bits");
  constexpr uint32_t NW = NT / WAVE;
  WaveAgg st;
  const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
  const uint4* sq = reinterpret_cast<const uint4*>(staging);
  if (T == 0) return;
  const uint32_t G = (T + WAVE - 1) / WAVE;  // groups of 64 tiles
  const uint32_t wpg = G < NW ? NW / G : 1;  // waves per group
  const uint32_t gstep = NW / wpg;           // groups between a wave's groups
  const uint32_t sub = w % wpg;
  if (w >= gstep * wpg) return;  // spare waves when NW is not a multiple of G
  // segment bounds of this lane's tile in group g (a clamped row past the end)
  auto bounds = [&](uint32_t g, uint32_t& lo, uint32_t& hi) {
    uint32_t t = g * WAVE + lane;
    t = t < T ? t : T - 1;
    const uint16_t* row = seg + (uint64_t)t * bstride;
    lo = row[b];
    hi = row[b + 1];
  };
  uint32_t g = w / wpg;
  uint32_t lo = 0, hi = 0;
  if (g < G) bounds(g, lo, hi);
  for (; g < G; g += gstep) {
    uint32_t nlo, nhi;
    bounds(g + gstep < G ? g + gstep : g, nlo, nhi);
    const uint32_t t = g * WAVE + lane;
    uint32_t e = hi < (uint32_t)TK ? hi : (uint32_t)TK;  // a segment never leaves its tile
    uint32_t s = lo < e ? lo : e;
    if (t >= T) s = e = 0;
    const uint32_t q0 = s >> 3;
    const uint32_t nq = e > s ? ((e + 7) >> 3) - q0 : 0;
    const uint32_t kmax = wave_max(nq);
    const uint64_t qb = nq ? (uint64_t)t * (TK / 8) + q0 : 0;
    const uint32_t qlast = nq ? nq - 1 : 0;
    for (uint32_t k0 = sub * BK_SQ; k0 < kmax; k0 += wpg * BK_SQ) {
      uint4 d[BK_SQ];
#pragma unroll
      for (int j = 0; j < BK_SQ; ++j) {
        const uint32_t k = k0 + j < qlast ? k0 + j : qlast;
        d[j] = sq[qb + k];
      }
#pragma unroll
      for (int j = 0; j < BK_SQ; ++j) {
        // valid keys of this quad: tile-local indices [s, e) within [q, q + 8)
        const int32_t q = (int32_t)((q0 + k0 + j) * 8);
        const int32_t lob = max((int32_t)s - q, 0), hib = min((int32_t)e - q, 8);
        const uint32_t qm = hib > lob ? ((1u << hib) - 1u) & ~((1u << lob) - 1u) : 0u;
        const uint32_t wds[4] = {d[j].x, d[j].y, d[j].z, d[j].w};
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const uint32_t x = (m & 1) ? (wds[m >> 1] >> 16) : (wds[m >> 1] & 0xFFFFu);
          bool ok = (qm >> m) & 1u;
          if (GM == GM_HALF) ok = ok && (x >> 15) == half;
          WaveGroups grp;
          const uint32_t n = wave_merge_count<AGG>(x, ok, st, grp);
          // lanes without a count issue nothing: as no-ops they would all hit
          // one word (masked keys, merged group members) and serialise
          if (n) {
            if (GM == GM_PACKED) {
              atomicAdd(&S.s[x >> 1], n << ((x & 1u) << 4));
            } else if (GM == GM_HALF) {
              atomicAdd(&S.s[x & 0x7FFFu], n);
            } else {
              atomicAdd(&S.s[x], n);
            }
          }
        }
      }
    }
    lo = nlo;
    hi = nhi;
  }
}

// Count of relative bin k on the packed path (no field wrapped).
template <typename SM>
__device__ __forceinline__ uint32_t packed_count(const SM& S, uint32_t k) {
  return (S.s[k >> 1] >> ((k & 1u) << 4)) & 0xFFFFu;
}

// Block sum over NT threads (result in every thread).  Ends with a barrier, so
// that S.red may be written by the next block operation at once: without it a
// fast wave could overwrite S.red while slower waves still read it, and the
// waves would then see different sums.
template <int NT, typename SM>
__device__ __forceinline__ uint64_t block_sum(SM& S, uint64_t x) {
  const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
  x = wave_sum(x);
  __syncthreads();
  if (lane == 0) S.red[w] = x;
  __syncthreads();
  uint64_t a = 0;
  for (uint32_t i = 0; i < NT / WAVE; ++i) a += S.red[i];
  __syncthreads();
  // the same in every lane: keep it in scalar registers
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Append fill items for this thread's bins: the thread owns NB consecutive bins
// starting at relative bin j0, whose counts come from count(j) and sum to len;
// o0 is the absolute position where its stretch starts.  The thread's bins lie
// in a span of output positions [sp0, sp1) (the run of a group of bins ending
// at bin klast) whose items start at index item0; threads may belong to
// different spans.
template <int NT, uint32_t NB, typename SM, typename CountF>
__device__ __forceinline__ void emit_items(SM& S, FillItem* __restrict__ items, uint32_t item0, int CL2,
                                           uint64_t sp0, uint64_t sp1, uint64_t hb, uint32_t j0, uint32_t nb_valid,
                                           uint64_t o0, uint64_t len, uint32_t klast, CountF count) {
  const uint32_t tid = threadIdx.x;
  const uint64_t C = 1ull << CL2;
  const uint64_t cb = sp0 >> CL2;
  // chunk starts c*C strictly inside the span and inside the run [o, o+h)
  auto starts = [&](uint64_t o, uint64_t h, uint64_t& lo, uint64_t& cntc) {
    lo = 0; cntc = 0;
    if (h > 0) {
      lo = (o + C - 1) >> CL2;
      if (lo < cb + 1) lo = cb + 1;
      const uint64_t hi = (o + h - 1) >> CL2;
      cntc = hi >= lo ? hi - lo + 1 : 0;
    }
  };
  // Only a thread whose stretch [o0, o0 + len) holds the span start or a chunk
  // start c*C (c > cb) has items to write; the others skip their bins.
  uint64_t o = o0;
  bool anylong = false;
  bool mine = false;
  {
    uint64_t lo, cntc;
    starts(o0, len, lo, cntc);
    mine = (len > 0) && (o0 == sp0 || cntc > 0);
  }
  if (mine) {
    for (uint32_t j = 0; j < NB; ++j) {
      const uint32_t i = j0 + j;
      const uint64_t h = i < nb_valid ? count(i) : 0u;
      if (h > 0 && o == sp0) {  // the span's first nonzero bin opens item 0
        FillItem it;
        it.p0 = sp0; it.p1 = ((cb + 1) << CL2) < sp1 ? ((cb + 1) << CL2) : sp1;
        it.o = o; it.k = (uint32_t)(hb + i); it.klast = klast;
        items[item0] = it;
      }
      uint64_t lo, cntc;
      starts(o, h, lo, cntc);
      if (cntc > 4) {
        anylong = true;  // written below by the whole block
      } else {
        for (uint64_t c = lo; c < lo + cntc; ++c) {
          FillItem it;
          it.p0 = c << CL2; it.p1 = ((c + 1) << CL2) < sp1 ? ((c + 1) << CL2) : sp1;
          it.o = o; it.k = (uint32_t)(hb + i); it.klast = klast;
          items[item0 + (c - cb)] = it;
        }
      }
      o += h;
    }
  }
  // runs that cross more than 4 chunk starts (rare): one bin per thread per
  // round through the long-run list, all threads writing the items
  if (!__syncthreads_or(anylong)) return;
  o = o0;
  for (uint32_t j = 0; j < NB; ++j) {
    const uint32_t i = j0 + j;
    const uint64_t h = (anylong && i < nb_valid) ? count(i) : 0u;
    uint64_t lo, cntc;
    starts(o, h, lo, cntc);
    bool pending = cntc > 4;
    while (__syncthreads_or(pending)) {
      if (tid == 0) S.n = 0;
      __syncthreads();
      if (pending) {
        const uint32_t slot = atomicAdd(&S.n, 1u);
        if (slot < BK_LRCAP) {
          // the entry carries its own span: spans differ between threads
          S.lr_o[slot] = o; S.lr_c[slot] = lo; S.lr_n[slot] = (uint32_t)cntc; S.lr_k[slot] = (uint32_t)(hb + i);
          S.lr_i[slot] = item0 + (uint32_t)(lo - cb); S.lr_e[slot] = sp1; S.lr_l[slot] = klast;
          pending = false;
        }
      }
      __syncthreads();
      const uint32_t nl = S.n < BK_LRCAP ? S.n : BK_LRCAP;
      for (uint32_t e2 = 0; e2 < nl; ++e2) {
        const uint64_t oo = S.lr_o[e2], cc = S.lr_c[e2], nn = S.lr_n[e2], ee = S.lr_e[e2];
        const uint32_t kk = S.lr_k[e2], ii = S.lr_i[e2], ll = S.lr_l[e2];
        for (uint64_t x = tid; x < nn; x += NT) {
          const uint64_t c = cc + x;
          FillItem it;
          it.p0 = c << CL2; it.p1 = ((c + 1) << CL2) < ee ? ((c + 1) << CL2) : ee;
          it.o = oo; it.k = kk; it.klast = ll;
          items[ii + (uint32_t)x] = it;
        }
      }
      __syncthreads();
    }
    o += h;
  }
}

// Reserve the items of span [sp0, sp1) (thread 0) and broadcast the first index.
template <typename SM>
__device__ __forceinline__ uint32_t reserve_items(SM& S, uint32_t* status, uint32_t* nitems, uint64_t sp0,
                                                  uint64_t sp1, uint32_t item_cap, int CL2) {
  const uint64_t C = 1ull << CL2;
  const uint64_t nit = sp1 > sp0 ? ((sp1 + C - 1) >> CL2) - (sp0 >> CL2) : 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t i0 = 0;
    if (nit) {
      i0 = atomicAdd(nitems, (uint32_t)nit);
      if ((uint64_t)i0 + nit > item_cap) { atomicOr(status, ST_INT_ITEMS); i0 = 0xFFFFFFFFu; }
    }
    S.item0 = i0;
  }
  __syncthreads();
  return S.item0;
}

// Bins per projection tile: fill items never walk more bins than this.
constexpr uint32_t PT_BINS = 1024;

// Project the counts held in S: the piece covers relative bins [0, pcnt) of
// absolute first bin hb, counts in S.s (uint32, or packed 16-bit fields when
// PACKED), and its run starts at output position base.  Each thread owns NB
// consecutive bins; a block scan of their sums tells it where its stretch
// starts.  Groups of PT_BINS bins (G = PT_BINS / NB threads, inside one wave)
// form tiles, each with its own span of output positions, so that no fill item
// walks more than PT_BINS bins; a second block scan numbers the tiles' items.
// Returns the piece's total.
template <int NT, uint32_t NB, bool PACKED, typename SM>
__device__ __forceinline__ uint64_t project_piece(SM& S, uint32_t* status, uint32_t* nitems, FillItem* items,
                                                  uint32_t item_cap, int CL2, uint64_t base, uint64_t hb,
                                                  uint32_t pcnt, uint32_t klast) {
  constexpr uint32_t G = PT_BINS / NB < (uint32_t)WAVE ? (PT_BINS / NB > 0 ? PT_BINS / NB : 1) : (uint32_t)WAVE;
  static_assert((G & (G - 1)) == 0, "tiles are a power of two of threads");
  const uint32_t tid = threadIdx.x, lane = lane_id();
  const uint32_t j0 = tid * NB;
  // the thread's NB bins, read in an order rotated by lane so that the lanes of
  // a wave hit different banks; bins at or beyond pcnt are never counted
  // (their keys are out of range), so their counters are zero
  uint32_t sum = 0;
  if constexpr (PACKED) {
    constexpr uint32_t NW = NB / 2;
#pragma unroll 8
    for (uint32_t w = 0; w < NW; ++w) {
      const uint32_t word = S.s[(j0 >> 1) + ((w + lane) & (NW - 1))];
      sum += (word & 0xFFFFu) + (word >> 16);
    }
  } else {
#pragma unroll 8
    for (uint32_t j = 0; j < NB; ++j) sum += S.s[j0 + ((j + lane) & (NB - 1))];
  }
  uint64_t tot;
  const uint64_t pre = block_exclusive_sum<NT>((uint64_t)sum, S.red, &tot);
  if (tot == 0) return 0;
  // the thread's tile: threads [lead, lead + G) of its wave
  const uint32_t lead = lane & ~(G - 1);
  const uint64_t ts = base + (uint64_t)__shfl((long long)pre, (int)lead, WAVE);
  uint64_t tsum = sum;
#pragma unroll
  for (uint32_t d = 1; d < G; d <<= 1) tsum += (uint64_t)__shfl_xor((long long)tsum, (int)d, WAVE);
  const uint64_t te = ts + tsum;
  const uint64_t C = 1ull << CL2;
  const uint64_t tnit = te > ts ? ((te + C - 1) >> CL2) - (ts >> CL2) : 0;
  uint64_t all_items;
  const uint64_t toff = block_exclusive_sum<NT>((uint64_t)(lane == lead ? tnit : 0ull), S.red, &all_items);
  const uint64_t tile_off = (uint64_t)__shfl((long long)toff, (int)lead, WAVE);
  const uint32_t tfirst = (tid - (lane - lead)) * NB;  // first relative bin of the tile
  const uint32_t tklast = (uint32_t)(hb + (tfirst + G * NB < pcnt ? tfirst + G * NB : pcnt) - 1);
  (void)klast;
  // reserve all the piece's items at once (thread 0) and broadcast the first
  __syncthreads();
  if (tid == 0) {
    uint32_t i0 = 0;
    if (all_items) {
      i0 = atomicAdd(nitems, (uint32_t)all_items);
      if ((uint64_t)i0 + all_items > item_cap) { atomicOr(status, ST_INT_ITEMS); i0 = 0xFFFFFFFFu; }
    }
    S.item0 = i0;
  }
  __syncthreads();
  const uint32_t item0 = S.item0;
  if (item0 == 0xFFFFFFFFu) return tot;
  const uint32_t my0 = item0 + (uint32_t)tile_off;
  if constexpr (PACKED) {
    auto count = [&](uint32_t i) -> uint32_t { return packed_count(S, i); };
    emit_items<NT, NB>(S, items, my0, CL2, ts, te, hb, j0, pcnt, base + pre, sum, tklast, count);
  } else {
    auto count = [&](uint32_t i) -> uint32_t { return S.s[i]; };
    emit_items<NT, NB>(S, items, my0, CL2, ts, te, hb, j0, pcnt, base + pre, sum, tklast, count);
  }
  return tot;
}

// ---------------------------------------------------------------------------
// Pass 2
// ---------------------------------------------------------------------------
// Bucket b of W = 2^LOG2W bins (T tiles): H receives bins [b*W, min((b+1)*W, U)).
// FULL also appends the fill items of the bucket's sorted run.  With W = 2^16
// the bucket is counted into packed 16-bit fields; a field that passed 0xFFFF
// shows up as a sum of all fields below the number of keys gathered (a wrap of
// a low field costs 65535, of a high field 65536), and the bucket is then
// counted again, exactly, in two halves of 2^15 bins with 32-bit counters.
template <int NT, int LOG2W, int AGG, bool HALIGNED, bool FULL, int TK>
__device__ __forceinline__ void bucket_body(BinSmem<NT, LOG2W>& S, const uint16_t* __restrict__ staging,
                                            const uint16_t* __restrict__ seg, uint32_t bstride, uint32_t T,
                                            uint64_t U, uint32_t* __restrict__ H, uint32_t* status,
                                            uint32_t* nitems, FillItem* __restrict__ items, uint32_t item_cap,
                                            int CL2, uint32_t b) {
  constexpr uint32_t W = 1u << LOG2W;
  using SM = BinSmem<NT, LOG2W>;
  const uint32_t tid = threadIdx.x;
  const uint64_t hb = (uint64_t)b * W;
  const uint32_t cnt = (uint32_t)(U - hb < W ? U - hb : W);
  const uint32_t klast = (uint32_t)(hb + cnt - 1);

  // where the bucket's run starts (keys of earlier buckets) and its length; the
  // pass also brings the segment bounds into the caches for the gather, whose
  // lanes visit the same tiles
  uint64_t mb = 0, mt = 0;
#pragma unroll 4
  for (uint32_t tt = tid; tt < T; tt += NT) {
    const uint16_t* row = seg + (uint64_t)tt * bstride;
    const uint32_t lo = row[b], hi = row[b + 1];
    mb += lo;
    mt += hi - lo;
  }
  const uint64_t base = block_sum<NT>(S, mb);
  const uint64_t total = block_sum<NT>(S, mt);
  for (uint32_t i = tid; i < SM::WORDS; i += NT) S.s[i] = 0;
  __syncthreads();
  bucket_gather<NT, LOG2W, AGG, SM::PACKED ? GM_PACKED : GM_DIRECT, TK>(S, staging, seg, bstride, T, b, 0);
  __syncthreads();

  if constexpr (!SM::PACKED) {
    // ---- W <= 2^15: 32-bit counters ----------------------------------------
    for (uint32_t i = tid; i < cnt; i += NT) H[hb + i] = S.s[i];
    if constexpr (FULL) {
      if (total) project_piece<NT, W / NT, false>(S, status, nitems, items, item_cap, CL2, base, hb, cnt, klast);
    }
    return;
  } else {
    // ---- packed fields: H from whole words, and the sum of the fields ------
    uint64_t fsum = 0;
    for (uint32_t wv = tid; wv < (cnt + 1) / 2; wv += NT) {
      const uint32_t k = 2 * wv;
      const uint32_t word = S.s[wv];
      const uint32_t c0 = word & 0xFFFFu, c1 = word >> 16;
      fsum += c0 + c1;
      if (HALIGNED && k + 1 < cnt) {
        *reinterpret_cast<uint2*>(H + hb + k) = make_uint2(c0, c1);
      } else {
        H[hb + k] = c0;
        if (k + 1 < cnt) H[hb + k + 1] = c1;
      }
    }
    if (block_sum<NT>(S, fsum) == total) {
      if constexpr (FULL) {
        if (total) project_piece<NT, W / NT, true>(S, status, nitems, items, item_cap, CL2, base, hb, cnt, klast);
      }
      return;
    }

    // ---- a field wrapped: two halves of 2^15 bins with 32-bit counters -----
    uint64_t hbase = base;  // where the current half's run starts
    for (uint32_t half = 0; half < 2; ++half) {
      const uint32_t hb0 = half << 15;
      if (hb0 >= cnt) break;
      const uint32_t hcnt = cnt - hb0 < (1u << 15) ? cnt - hb0 : (1u << 15);
      __syncthreads();
      for (uint32_t i = tid; i < SM::WORDS; i += NT) S.s[i] = 0;
      if (tid == 0) S.n = 0;
      __syncthreads();
      bucket_gather<NT, LOG2W, AGG, GM_HALF, TK>(S, staging, seg, bstride, T, b, half);
      __syncthreads();
      for (uint32_t i = tid; i < hcnt; i += NT) H[hb + hb0 + i] = S.s[i];
      if constexpr (FULL) {
        hbase += project_piece<NT, (1u << 15) / NT, false>(S, status, nitems, items, item_cap, CL2, hbase,
                                                           hb + hb0, hcnt, klast);
      }
    }
  }
}

template <int AGG, bool HALIGNED, bool FULL>
__global__ __launch_bounds__(PART_NT) void k_bucket(const uint16_t* __restrict__ staging,
                                                    const uint16_t* __restrict__ seg, uint32_t bstride,
                                                    uint32_t T, uint32_t B, uint64_t U, uint32_t* __restrict__ H,
                                                    Ctl* ctl, FillItem* __restrict__ items, uint32_t item_cap,
                                                    int CL2) {
  __shared__ __align__(16) BinSmem<PART_NT, PART_LOG2W> S;
  // XCD-aware bucket order: blocks are dispatched round-robin over 8 XCDs
  uint32_t b = blockIdx.x;
  if ((B & 7u) == 0) b = (blockIdx.x & 7u) * (B >> 3) + (blockIdx.x >> 3);
  bucket_body<PART_NT, PART_LOG2W, AGG, HALIGNED, FULL, PART_TK>(S, staging, seg, bstride, T, U, H, &ctl->status,
                                                        &ctl->nitems, items, item_cap, CL2, b);
}

// ---------------------------------------------------------------------------
// Row sum + projection of a small universe (U <= 2^16) in one workgroup
// ---------------------------------------------------------------------------
// Sums nrows partial rows (row r at rows + r*row_stride) into H (skipped when
// H_out is null: rows already is H) and, FULL, appends the fill items of the
// whole output, piece by piece of P = min(W, 2^15) bins.
template <int NT, int LOG2W, bool FULL>
__device__ __forceinline__ void rows_body(BinSmem<NT, LOG2W>& S, const uint32_t* __restrict__ rows, uint32_t nrows,
                                          uint64_t row_stride, uint32_t* __restrict__ H_out, uint32_t U,
                                          uint32_t* status, uint32_t* nitems, FillItem* __restrict__ items,
                                          uint32_t item_cap, int CL2) {
  constexpr uint32_t P = LOG2W >= 15 ? (1u << 15) : (1u << LOG2W);
  const uint32_t tid = threadIdx.x;
  uint64_t pbase = 0;
  for (uint32_t p0 = 0; p0 < U; p0 += P) {
    const uint32_t pcnt = U - p0 < P ? U - p0 : P;
    __syncthreads();  // S.s of the previous piece is no longer read
    for (uint32_t i = tid; i < P; i += NT) {
      uint32_t a = 0;
      if (i < pcnt) {
        const uint32_t* r = rows + p0 + i;
#pragma unroll 4
        for (uint32_t j = 0; j < nrows; ++j) a += r[(uint64_t)j * row_stride];
        if (H_out) H_out[p0 + i] = a;
      }
      S.s[i] = a;
    }
    __syncthreads();
    if constexpr (FULL) {
      const uint32_t klast = p0 + pcnt - 1;
      pbase += project_piece<NT, P / NT, false>(S, status, nitems, items, item_cap, CL2, pbase, p0, pcnt, klast);
    }
  }
}

}  // namespace ds
