// U-range-partitioned ingestion and projection for universes larger than one
// workgroup's LDS.
//
// The paper leaves large universes to a "hierarchical" scheme it lists as future
// work (Sec. 16 and Sec. 17); this two-pass design is ours.  The universe is cut
// into B buckets of W = 2^16 consecutive keys (bucket of x = x >> 16).
//
// Pass 1 (k_partition): workgroup t takes tile t of TK = 8192 keys, counts them
// per bucket, scans the counts and places every key at a cursor of its bucket
// (LDS atomics: with few buckets into per-lane copies of each bucket's counter,
// and where many lanes share a counter after the wavefront equality merge).
// It writes the tile's keys
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
constexpr uint32_t SPLIT_SLOTS = 16;  // heavy buckets that may be split between workgroups in one call
constexpr uint32_t HEAVY_MAX = 512;   // heavy buckets ranked for the slots (the first ones in bucket order)

// Rows of bucket-total counters the partition adds into (tile t into row t mod
// rows): enough rows to spread the atomics, at most 8192 counters in all.
__host__ __device__ constexpr uint32_t colsum_rows(uint32_t B) {
  return B <= 256 ? 16u : (B <= 1024 ? 4u : (B <= 4096 ? 2u : 1u));
}

// Heavy-bucket splitting on the partitioned path.  The partition adds each
// tile's bucket counts into colsum (row tile mod rows); the bucket pass reads
// the totals back and lets several workgroups count a heavy bucket, each into
// the bucket's scratch row of 32-bit counters.  colsum, done and scratch are
// cleared before the partition runs.
struct SplitPlan {
  uint32_t* colsum;   // rows x B bucket-total counters
  uint32_t rows;      // colsum_rows(B)
  uint32_t* done;     // per slot: parts finished
  uint32_t* scratch;  // SPLIT_SLOTS rows of PART_W counters
  uint64_t chunk;     // keys per part of a split bucket
  uint32_t X;         // extra workgroups of the bucket pass
};

// ---------------------------------------------------------------------------
// Pass 1
// ---------------------------------------------------------------------------
// Copies of each bucket's counter a tile keeps when it has few buckets: with
// C = 2^lc copies, lane l counts into copy l mod C, so the 64 lanes of a slot
// spread over up to 64 counters instead of B.  The copies of bucket b are
// counters b*C .. b*C + C - 1, consecutive, so the exclusive scan over all of
// them still places every bucket's keys together (a copy's cursor starts
// where the previous copy's keys end), and bucket b starts at counter b*C.
__device__ __forceinline__ uint32_t part_copies_log2(uint32_t B) {
  const uint32_t lb = B > 1 ? 32u - (uint32_t)__clz(B - 1) : 0u;  // ceil(log2 B)
  return lb < 6 ? 6 - lb : 0;
}

template <int NT, int BMAXT, int TK>
struct PartSmem {
  uint32_t cnt[BMAXT + 1];
  __align__(16) uint16_t stage[TK];
  uint32_t scan_tmp[NT / WAVE + 1];
};

// Tile `tile` of TK keys (NT threads; TK <= 65536 so segment starts fit in uint16).  seg: T rows of `bstride` uint16
// (bstride >= B + 1, multiple of 8).  Invalid keys are parked as 0xFFFFFFFF
// (U <= 2^29 here, so no valid key has that value).  Bucket of x: x >> LOG2W.
// plan (optional): the tile adds its bucket counts into counter row tile mod
// plan->rows.
template <int NT, int BMAXT, int AGG, bool ALIGNED, int LOG2W, int TK>
__device__ __forceinline__ void partition_tile(PartSmem<NT, BMAXT, TK>& S, const uint32_t* __restrict__ keys, uint64_t n,
                                               uint32_t umax, uint32_t B, uint16_t* __restrict__ staging,
                                               uint16_t* __restrict__ seg, uint32_t bstride, uint32_t* status,
                                               uint32_t tile, const SplitPlan* plan, uint32_t lo = 0) {
  constexpr int GPT = TK / 4 / NT;  // key groups of 4 per thread
  static_assert(GPT >= 1, "a tile gives every thread at least one group");
  constexpr uint32_t WM = (1u << LOG2W) - 1;
  const uint32_t tid = threadIdx.x;
  const uint64_t tb = (uint64_t)tile * TK;
  const uint64_t te = tb + TK < n ? tb + TK : n;

  // counters: B buckets, times 2^lc copies on a tile without merging
  const uint32_t lc = part_copies_log2(B);
  for (uint32_t i = tid; i <= (B << lc); i += NT) S.cnt[i] = 0;

  uint32_t v[GPT][4];
  bool bad = false;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const uint32_t c = load_group<ALIGNED>(keys, tb + ((uint64_t)u * NT + tid) * 4, te, v[u], lo);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool valid = (uint32_t)i < c;
      const bool ok = valid && v[u][i] <= umax;
      bad |= valid && !ok;
      if (!ok) v[u][i] = 0xFFFFFFFFu;
    }
  }
  // Equality merging pays only where many lanes share a counter: a tile takes
  // it when some wave finds 8 or more of its first 64 keys (one per lane) on
  // the counter (bucket and copy) of its lowest lane's key.  Merging tiles
  // count each bucket in one counter, the others in 2^lc copies.  Either way
  // every count is exact.
  const uint32_t cmask = (1u << lc) - 1;
  bool crowd = false;
  if constexpr (AGG != 0) {
    const uint32_t x0 = v[0][0];
    const uint32_t ci = x0 != 0xFFFFFFFFu ? ((x0 >> LOG2W) << lc) | (lane_id() & cmask) : 0xFFFFFFFFu;
    const uint32_t lead = __builtin_amdgcn_readfirstlane(ci);
    crowd = lead != 0xFFFFFFFFu && __popcll(__ballot(ci == lead)) >= 8;
  }
  const bool merge = __syncthreads_or(crowd);
  const uint32_t cl = merge ? 0u : lc;  // copies of this tile: 2^cl
  const uint32_t cm = (1u << cl) - 1, nc = B << cl;
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
        const uint32_t x = v[u][i];
        if (x != 0xFFFFFFFFu) atomicAdd(&S.cnt[((x >> LOG2W) << cl) | (lane_id() & cm)], 1u);
      }
    }
  }
  if (__syncthreads_or(bad) && tid == 0) atomicOr(status, ST_RANGE);

  // exclusive scan of the nc+1 counters (counter nc stays 0, so the total is
  // the number of valid keys); each thread owns a run of CPT counters.
  // Bucket b starts at counter b << cl; counter nc gives seg[B].
  static_assert(BMAXT >= 64, "the copies of a few buckets fit the counters");
  if (plan != nullptr) {
    // bucket totals: one global add per nonzero bucket (its copies summed here)
    for (uint32_t b = tid; b < B; b += NT) {
      uint32_t t = 0;
      for (uint32_t c = 0; c <= cm; ++c) t += S.cnt[(b << cl) + c];
      if (t) atomicAdd(&plan->colsum[(tile & (plan->rows - 1)) * B + b], t);
    }
  }
  constexpr int CPT = (BMAXT + 1 + NT - 1) / NT;
  uint32_t loc[CPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    loc[j] = i <= nc ? S.cnt[i] : 0;
    sum += loc[j];
  }
  uint32_t total;
  uint32_t pre = block_exclusive_sum<NT>(sum, S.scan_tmp, &total);
  uint16_t* srow = seg + (uint64_t)tile * bstride;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    if (i <= nc) {
      S.cnt[i] = pre;
      if ((i & cm) == 0) srow[i >> cl] = (uint16_t)pre;
    }
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
          if (x != 0xFFFFFFFFu) pos[u][i] = atomicAdd(&S.cnt[((x >> LOG2W) << cl) | (lane_id() & cm)], 1u);
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

template <int BMAXT, int AGG, bool ALIGNED>
__global__ __launch_bounds__(P1_NT) void k_partition(const uint32_t* __restrict__ keys, uint64_t n,
                                                     uint32_t umax, uint32_t B,
                                                     uint16_t* __restrict__ staging,
                                                     uint16_t* __restrict__ seg, uint32_t bstride, Ctl* ctl,
                                                     SplitPlan plan, uint32_t lo) {
  __shared__ PartSmem<P1_NT, BMAXT, PART_TK> S;
  partition_tile<P1_NT, BMAXT, AGG, ALIGNED, PART_LOG2W, PART_TK>(S, keys, n, umax, B, staging, seg, bstride,
                                                                 &ctl->status, blockIdx.x, &plan, lo);
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
  __align__(16) uint32_t s[WORDS];
  uint32_t evflag[PACKED ? 65536 / 32 : 1];
  uint32_t ev[PACKED ? LDS16_EVCAP : 1];
  uint32_t nev;
  uint32_t lr_k[BK_LRCAP], lr_n[BK_LRCAP], lr_l[BK_LRCAP], lr_i[BK_LRCAP];
  uint64_t lr_o[BK_LRCAP], lr_c[BK_LRCAP], lr_e[BK_LRCAP];
  uint64_t red[NT / WAVE + 1];
  uint32_t n, item0;
};

enum GatherMode { GM_PACKED, GM_PACKED_HOT, GM_PACKED_HOT2, GM_HALF, GM_DIRECT };

// GM_PACKED_HOT (GM_PACKED_HOT2): as GM_PACKED, except that each wave counts
// one (two) candidate keys in registers (each lane adds its matches to acc; no
// LDS atomic for them) and flushes a candidate's count into the bucket's hot
// table -- pairs (key, count) in the packed layout's event-log storage (S.ev,
// unused on this path), numbered by S.nev -- when the candidate changes and
// when the gather ends.  Every 16th slot looks for a group of AGG_HOT_MIN or
// more lanes on one key that is no candidate; a group larger than the
// (smaller) candidate's group in that slot replaces that candidate.  A hot key
// therefore never passes through a 16-bit field.  The second candidate costs
// every key a compare, so a bucket is gathered with one, and again with two
// only if another key wrapped a field.
constexpr uint32_t BK_HOTCAP = LDS16_EVCAP / 2;  // hot table entries

struct HotGather {
  uint32_t hk[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};  // wave-uniform; bucket-relative keys are below 2^16
  uint32_t acc[2] = {0, 0};                      // per lane
  uint32_t slot = 15;                            // wave-uniform
};

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
// counted.  Only tiles [t0, t1) are visited; returns the number of keys in the
// segments this thread owned (each segment belongs to one lane of one wave).
// Count the 8 keys of quad d (tile-local key indices [8q, 8q + 8)) that lie in
// [s, e) (and, GM_HALF, in half `half`) into S, after the wave merge.
template <int NT, int LOG2W>
__device__ __forceinline__ void hot_flush(BinSmem<NT, LOG2W>& S, HotGather& h, int j) {
  const uint32_t c = __builtin_amdgcn_readfirstlane(wave_sum(h.acc[j]));
  h.acc[j] = 0;
  if (c && lane_id() == 0) {
    const uint32_t i = atomicAdd(&S.nev, 1u);
    if (i < BK_HOTCAP) {
      S.ev[2 * i] = h.hk[j];
      S.ev[2 * i + 1] = c;
    }
  }
}

// Total count of hot bin k (relative) from the bucket's merged hot table:
// after the merge each key has one live entry holding field + table counts.
template <typename SM>
__device__ __forceinline__ uint32_t hot_total(const SM& S, uint32_t nhot, uint32_t k) {
  for (uint32_t i = 0; i < nhot; ++i)
    if (S.ev[2 * i] == k) return S.ev[2 * i + 1];
  return 0;
}

template <typename SM>
__device__ __forceinline__ bool hot_flag(const SM& S, uint32_t k) {
  return (S.evflag[k >> 5] >> (k & 31)) & 1u;
}

template <int NT, int LOG2W, int AGG, GatherMode GM>
__device__ __forceinline__ void count_quad(BinSmem<NT, LOG2W>& S, const uint4& d, int32_t q8, uint32_t s, uint32_t e,
                                           uint32_t half, WaveAgg& st, HotGather& h) {
  const int32_t lob = max((int32_t)s - q8, 0), hib = min((int32_t)e - q8, 8);
  const uint32_t qm = hib > lob ? ((1u << hib) - 1u) & ~((1u << lob) - 1u) : 0u;
  const uint32_t wds[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const uint32_t x = (m & 1) ? (wds[m >> 1] >> 16) : (wds[m >> 1] & 0xFFFFu);
    bool ok = (qm >> m) & 1u;
    if constexpr (GM == GM_PACKED_HOT || GM == GM_PACKED_HOT2) {
      constexpr bool TWO = GM == GM_PACKED_HOT2;
      const bool eq0 = ok && x == h.hk[0], eq1 = TWO && ok && x == h.hk[1];
      h.acc[0] += eq0 ? 1u : 0u;
      if constexpr (TWO) h.acc[1] += eq1 ? 1u : 0u;
      bool act = ok && !eq0 && !eq1;
      if (((++h.slot) & 15u) == 0u) {
        const uint64_t am = __ballot(act);
        if (am) {
          const uint32_t ll = (uint32_t)__ffsll((unsigned long long)am) - 1;
          const uint32_t lk = (uint32_t)__builtin_amdgcn_readlane((int)x, (int)ll);
          const bool e2 = act && x == lk;
          const uint32_t c2 = (uint32_t)__popcll(__ballot(e2));
          const uint32_t n0 = (uint32_t)__popcll(__ballot(eq0));
          const uint32_t n1 = TWO ? (uint32_t)__popcll(__ballot(eq1)) : 0xFFFFFFFFu;
          const int jm = n1 < n0 ? 1 : 0;  // the candidate with the smaller group here
          if (c2 >= AGG_HOT_MIN && c2 > (jm ? n1 : n0)) {
            hot_flush(S, h, jm);
            h.hk[jm] = lk;
            h.acc[jm] = e2 ? 1u : 0u;
            act = act && !e2;
          }
        }
      }
      if (act) atomicAdd(&S.s[x >> 1], 1u << ((x & 1u) << 4));
      continue;
    }
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

// Bucket b's segments of fewer than 64 tiles: the waves take the tiles (NW / T
// waves per tile when there are fewer tiles than waves) and all 64 lanes of a
// wave walk one segment, BK_SQ 16-byte quads per lane per step, the step count
// uniform over the wave (lanes past the segment's end reread its last quad,
// masked out).  With one lane per tile, as below, such a bucket would keep at
// most T lanes of each wave busy.
template <int NT, int LOG2W, int AGG, GatherMode GM, int TK>
__device__ __forceinline__ uint32_t bucket_gather_few(BinSmem<NT, LOG2W>& S, const uint16_t* __restrict__ staging,
                                                      const uint16_t* __restrict__ seg, uint32_t bstride, uint32_t t0,
                                                      uint32_t T, uint32_t b, uint32_t half) {
  constexpr uint32_t NW = NT / WAVE;
  WaveAgg st;
  HotGather h;
  const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
  const uint4* sq = reinterpret_cast<const uint4*>(staging);
  const uint32_t wpt = T < NW ? NW / T : 1;  // waves per tile
  const uint32_t tstep = NW / wpt;           // tiles between a wave's tiles
  const uint32_t sub = w % wpt;
  if (w >= tstep * wpt) return 0;  // spare waves when NW is not a multiple of T
  uint32_t counted = 0;
  for (uint32_t i = w / wpt; i < T; i += tstep) {  // wave-uniform
    const uint32_t t = t0 + i;
    const uint16_t* row = seg + (uint64_t)t * bstride;
    const uint32_t e = row[b + 1] < (uint32_t)TK ? row[b + 1] : (uint32_t)TK;
    const uint32_t s = row[b] < e ? row[b] : e;
    if (sub == 0 && lane == 0) counted += e - s;
    if (e <= s) continue;
    const uint32_t q0 = s >> 3, q1 = (e + 7) >> 3;  // quads [q0, q1) of the tile
    const uint64_t tq = (uint64_t)t * (TK / 8);
    constexpr uint32_t CH = WAVE * BK_SQ;  // quads per wave step
    for (uint32_t c0 = q0 + sub * CH; c0 < q1; c0 += wpt * CH) {  // wave-uniform
      uint4 d[BK_SQ];
#pragma unroll
      for (int j = 0; j < BK_SQ; ++j) {
        const uint32_t q = c0 + j * WAVE + lane;
        d[j] = sq[tq + (q < q1 ? q : q1 - 1)];
      }
#pragma unroll
      for (int j = 0; j < BK_SQ; ++j) {
        const uint32_t q = c0 + j * WAVE + lane;
        // a reread quad counts nothing: its window [8q, 8q + 8) lies past e
        count_quad<NT, LOG2W, AGG, GM>(S, d[j], (int32_t)(q * 8), s, e, half, st, h);
      }
    }
  }
  if constexpr (GM == GM_PACKED_HOT || GM == GM_PACKED_HOT2) {  // the wave's last candidates
    hot_flush(S, h, 0);
    if constexpr (GM == GM_PACKED_HOT2) hot_flush(S, h, 1);
  }
  return counted;
}

template <int NT, int LOG2W, int AGG, GatherMode GM, int TK>
__device__ __forceinline__ uint32_t bucket_gather(BinSmem<NT, LOG2W>& S, const uint16_t* __restrict__ staging,
                                                  const uint16_t* __restrict__ seg, uint32_t bstride, uint32_t t0,
                                                  uint32_t t1, uint32_t b, uint32_t half) {
  static_assert(TK % 8 == 0 && TK <= 32768, "tile-local key indices and quad offsets fit 16 bits");
  constexpr uint32_t NW = NT / WAVE;
  WaveAgg st;
  HotGather h;
  const uint32_t lane = lane_id(), w = threadIdx.x / WAVE;
  const uint4* sq = reinterpret_cast<const uint4*>(staging);
  uint32_t counted = 0;
  if (t1 <= t0) return 0;
  const uint32_t T = t1 - t0;               // tiles t0 + i, i < T
  if (T < WAVE) return bucket_gather_few<NT, LOG2W, AGG, GM, TK>(S, staging, seg, bstride, t0, T, b, half);
  const uint32_t G = (T + WAVE - 1) / WAVE;  // groups of 64 tiles
  const uint32_t wpg = G < NW ? NW / G : 1;  // waves per group
  const uint32_t gstep = NW / wpg;           // groups between a wave's groups
  const uint32_t sub = w % wpg;
  if (w >= gstep * wpg) return 0;  // spare waves when NW is not a multiple of G
  // segment bounds of this lane's tile in group g (a clamped row past the end)
  auto bounds = [&](uint32_t g, uint32_t& lo, uint32_t& hi) {
    uint32_t i = g * WAVE + lane;
    i = i < T ? i : T - 1;
    const uint16_t* row = seg + (uint64_t)(t0 + i) * bstride;
    lo = row[b];
    hi = row[b + 1];
  };
  uint32_t g = w / wpg;
  uint32_t lo = 0, hi = 0;
  if (g < G) bounds(g, lo, hi);
  for (; g < G; g += gstep) {
    uint32_t nlo, nhi;
    bounds(g + gstep < G ? g + gstep : g, nlo, nhi);
    const uint32_t i = g * WAVE + lane;
    const uint32_t t = t0 + i;
    uint32_t e = hi < (uint32_t)TK ? hi : (uint32_t)TK;  // a segment never leaves its tile
    uint32_t s = lo < e ? lo : e;
    if (i >= T) s = e = 0;
    if (sub == 0) counted += e - s;  // waves sharing a group count its keys once
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
        count_quad<NT, LOG2W, AGG, GM>(S, d[j], (int32_t)((q0 + k0 + j) * 8), s, e, half, st, h);
      }
    }
    lo = nlo;
    hi = nhi;
  }
  if constexpr (GM == GM_PACKED_HOT || GM == GM_PACKED_HOT2) {  // the wave's last candidates
    hot_flush(S, h, 0);
    if constexpr (GM == GM_PACKED_HOT2) hot_flush(S, h, 1);
  }
  return counted;
}

// Count of relative bin k on the packed path (no field wrapped).
template <typename SM>
__device__ __forceinline__ uint32_t packed_count(const SM& S, uint32_t k) {
  return (S.s[k >> 1] >> ((k & 1u) << 4)) & 0xFFFFu;
}


// Append fill items for this thread's bins: the thread owns NB consecutive bins
// starting at relative bin j0, whose counts come from count(j) and sum to len;
// o0 is the absolute position where its stretch starts.  The thread's bins lie
// in a span of output positions [sp0, sp1) (the run of a group of bins ending
// at bin klast) whose items start at index item0; threads may belong to
// different spans.  PAIRS: the counts are packed 16-bit pairs (bin i in word
// i / 2) and j0, NB are even, so the walk reads one word per two bins.
template <int NT, uint32_t NB, bool PAIRS, typename SM, typename CountF>
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
    // pn: the first chunk start c*C (c > cb) at or after o.  A bin [o, o + h)
    // has items to write only if it opens the span (o == sp0) or reaches pn;
    // every other bin just advances o.
    auto next_start = [&](uint64_t x) -> uint64_t {
      const uint64_t c = (x + C - 1) >> CL2;
      return (c > cb + 1 ? c : cb + 1) << CL2;
    };
    uint64_t pn = next_start(o);
    // bin i with count h: write its items if it has any, and advance o
    auto visit = [&](uint32_t i, uint64_t h) {
      if (h > 0 && (o == sp0 || o + h > pn)) {
        if (o == sp0) {  // the span's first nonzero bin opens item 0
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
        pn = next_start(o);
      } else {
        o += h;
      }
    };
    if constexpr (PAIRS) {
      // o >= sp0 throughout (the stretch starts inside its span), so a pair
      // with neither o == sp0 nor o + h0 + h1 > pn holds no item start
      for (uint32_t j = 0; j < NB; j += 2) {
        const uint32_t i = j0 + j;
        const uint32_t word = i < nb_valid ? S.s[i >> 1] : 0u;
        const uint64_t h0 = word & 0xFFFFu, h1 = i + 1 < nb_valid ? (word >> 16) : 0u;
        if (h0 + h1 > 0 && (o == sp0 || o + h0 + h1 > pn)) {
          visit(i, h0);
          visit(i + 1, h1);
        } else {
          o += h0 + h1;
        }
      }
    } else {
      for (uint32_t j = 0; j < NB; ++j) {
        const uint32_t i = j0 + j;
        visit(i, i < nb_valid ? count(i) : 0u);
      }
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
                                                  uint32_t pcnt, uint32_t klast, uint32_t nhot = 0) {
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
    if (nhot) {
      // hot bins: their merged totals in place of their fields
      for (uint32_t j = 0; j < NB; ++j)
        if (hot_flag(S, j0 + j)) sum += hot_total(S, nhot, j0 + j) - packed_count(S, j0 + j);
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
    if (nhot) {
      auto count = [&](uint32_t i) -> uint32_t {
        return hot_flag(S, i) ? hot_total(S, nhot, i) : packed_count(S, i);
      };
      emit_items<NT, NB, false>(S, items, my0, CL2, ts, te, hb, j0, pcnt, base + pre, sum, tklast, count);
    } else {
      auto count = [&](uint32_t i) -> uint32_t { return packed_count(S, i); };
      emit_items<NT, NB, (NB % 2 == 0)>(S, items, my0, CL2, ts, te, hb, j0, pcnt, base + pre, sum, tklast, count);
    }
  } else {
    auto count = [&](uint32_t i) -> uint32_t { return S.s[i]; };
    emit_items<NT, NB, false>(S, items, my0, CL2, ts, te, hb, j0, pcnt, base + pre, sum, tklast, count);
  }
  return tot;
}

// ---------------------------------------------------------------------------
// Pass 2
// ---------------------------------------------------------------------------
// Where bucket b's sorted run starts (the keys of buckets before b: the sum of
// seg[t][b] over the tiles) and how many keys it holds.  Result in every thread.
template <int NT, typename SM>
__device__ __forceinline__ void bucket_extent(SM& S, const uint16_t* __restrict__ seg, uint32_t bstride, uint32_t T,
                                              uint32_t b, uint64_t* base, uint64_t* total) {
  uint64_t mb = 0, mt = 0;
#pragma unroll 4
  for (uint32_t t = threadIdx.x; t < T; t += NT) {
    const uint16_t* row = seg + (uint64_t)t * bstride;
    const uint32_t lo = row[b], hi = row[b + 1];
    mb += lo;
    mt += hi - lo;
  }
  *base = block_sum<NT>(S, mb);
  *total = block_sum<NT>(S, mt);
}

// One part of bucket b: its segments in tiles [t0, t1), part p of P.  With
// P == 1 the part is the whole bucket and writes H with plain stores; with
// P > 1 (a heavy bucket) every part adds its counts into a cleared row of
// 32-bit scratch counters with global atomics, and the part that finishes last
// copies the row into H and projects the bucket from it.  base: keys of the
// buckets before b.
struct BucketPart {
  uint32_t b, t0, t1, P;
  uint64_t base;
  uint32_t* acc;   // P > 1: the bucket's scratch row
  uint32_t* done;  // P > 1: parts finished so far (starts at 0)
};

// Bins [lo, lo + len) of LDS counters into H[hb + lo + ...]: stored, or (add)
// added where nonzero.  PACKED_SRC reads bin j from the 16-bit field j of the
// packed words, else from word j - lo0 (32-bit counters of a piece starting at
// lo0).
template <int NT, bool PACKED_SRC, bool HALIGNED, typename SM>
__device__ __forceinline__ void emit_bins(const SM& S, uint32_t* __restrict__ H, uint64_t hb, uint32_t lo0,
                                          uint32_t len, bool add, uint32_t nhot = 0) {
  const uint32_t tid = threadIdx.x;
  if constexpr (PACKED_SRC) {
    // len bins from bin 0, two per word; with nhot (not add) the flagged hot
    // bins take their merged totals instead of their fields
    for (uint32_t wv = tid; wv < (len + 1) / 2; wv += NT) {
      const uint32_t k = 2 * wv;
      const uint32_t word = S.s[wv];
      uint32_t c0 = word & 0xFFFFu, c1 = word >> 16;
      if constexpr (SM::PACKED) {
        if (nhot && ((S.evflag[k >> 5] >> (k & 31)) & 3u)) {
          if (hot_flag(S, k)) c0 = hot_total(S, nhot, k);
          if (hot_flag(S, k + 1)) c1 = hot_total(S, nhot, k + 1);
        }
      }
      if (add) {
        if (c0) atomicAdd(&H[hb + k], c0);
        if (c1 && k + 1 < len) atomicAdd(&H[hb + k + 1], c1);
      } else if (HALIGNED && k + 1 < len) {
        *reinterpret_cast<uint2*>(H + hb + k) = make_uint2(c0, c1);
      } else {
        H[hb + k] = c0;
        if (k + 1 < len) H[hb + k + 1] = c1;
      }
    }
  } else {
    for (uint32_t i = tid; i < len; i += NT) {
      const uint32_t c = S.s[i];
      if (add) {
        if (c) atomicAdd(&H[hb + lo0 + i], c);
      } else {
        H[hb + lo0 + i] = c;
      }
    }
  }
}

// Bucket b of W = 2^LOG2W bins: H receives bins [b*W, min((b+1)*W, U)), and
// FULL also appends the fill items of the bucket's sorted run.  With W = 2^16
// the bucket is counted into packed 16-bit fields; a field that passed 0xFFFF
// shows up as a sum of all fields below the number of keys gathered (a wrap of
// a low field costs 65535, of a high field 65536), and the part is then
// counted again, exactly, in two halves of 2^15 bins with 32-bit counters.
template <int NT, int LOG2W, int AGG, bool HALIGNED, bool FULL, int TK>
__device__ __forceinline__ void bucket_body(BinSmem<NT, LOG2W>& S, const uint16_t* __restrict__ staging,
                                            const uint16_t* __restrict__ seg, uint32_t bstride, uint64_t U,
                                            uint32_t* __restrict__ H, uint32_t* status, uint32_t* nitems,
                                            FillItem* __restrict__ items, uint32_t item_cap, int CL2,
                                            const BucketPart& bp) {
  constexpr uint32_t W = 1u << LOG2W;
  using SM = BinSmem<NT, LOG2W>;
  const uint32_t tid = threadIdx.x;
  const uint32_t b = bp.b;
  const uint64_t hb = (uint64_t)b * W;
  const uint32_t cnt = (uint32_t)(U - hb < W ? U - hb : W);
  const uint32_t klast = (uint32_t)(hb + cnt - 1);
  const bool split = bp.P > 1;

  static_assert(SM::WORDS % 4 == 0, "16-byte clears");
  for (uint32_t i = tid; i < SM::WORDS / 4; i += NT) reinterpret_cast<uint4*>(S.s)[i] = make_uint4(0, 0, 0, 0);
  if constexpr (SM::PACKED) {
    for (uint32_t i = tid; i < 65536 / 32; i += NT) S.evflag[i] = 0;  // hot-bin flags
    if (tid == 0) S.nev = 0;                                          // hot table entries
  }
  __syncthreads();
  const uint32_t mine = bucket_gather<NT, LOG2W, AGG, SM::PACKED ? GM_PACKED_HOT : GM_DIRECT, TK>(
      S, staging, seg, bstride, bp.t0, bp.t1, b, 0);
  // the block sums end with barriers: every LDS count and hot entry is in place afterwards
  const uint64_t gathered = block_sum<NT>(S, (uint64_t)mine);

  // a split part adds into its bucket's scratch row instead of H
  uint32_t* const dst = split ? bp.acc : H;
  const uint64_t dhb = split ? 0 : hb;
  if constexpr (!SM::PACKED) {
    // ---- W <= 2^15: 32-bit counters ----------------------------------------
    emit_bins<NT, false, HALIGNED>(S, dst, dhb, 0, cnt, split);
    if constexpr (FULL) {
      if (!split && gathered)
        project_piece<NT, W / NT, false>(S, status, nitems, items, item_cap, CL2, bp.base, hb, cnt, klast);
    }
  } else {
    // The hot keys counted in registers sit in the hot table (nhot entries;
    // a table that overflowed lost entries, and the bucket is counted again).
    // The fields hold the other keys: fewer than 2^16 keys cannot wrap one,
    // otherwise the fields must sum to the keys gathered less the table's.
    auto check = [&](uint32_t& nhot) -> bool {
      const uint32_t nev = S.nev;
      nhot = nev < BK_HOTCAP ? nev : BK_HOTCAP;
      bool ok = nev <= BK_HOTCAP;
      if (ok && gathered > 0xFFFFu) {
        uint64_t fsum = 0;
        for (uint32_t wv = tid; wv < SM::WORDS; wv += NT) {
          const uint32_t word = S.s[wv];
          fsum += (word & 0xFFFFu) + (word >> 16);
        }
        for (uint32_t i = tid; i < nhot; i += NT) fsum += S.ev[2 * i + 1];
        ok = block_sum<NT>(S, fsum) == gathered;
      }
      return ok;
    };
    uint32_t nhot = 0;
    bool clean = check(nhot);
    if (!clean) {
      // a second key wrapped a field: gather again with two candidates per wave
      __syncthreads();
      for (uint32_t i = tid; i < SM::WORDS / 4; i += NT) reinterpret_cast<uint4*>(S.s)[i] = make_uint4(0, 0, 0, 0);
      if (tid == 0) S.nev = 0;
      __syncthreads();
      bucket_gather<NT, LOG2W, AGG, GM_PACKED_HOT2, TK>(S, staging, seg, bstride, bp.t0, bp.t1, b, 0);
      __syncthreads();
      clean = check(nhot);
    }
    if (clean && nhot > 0 && split) {
      // ---- a part with hot keys: fields and table entries all added -------
      emit_bins<NT, true, HALIGNED>(S, dst, dhb, 0, cnt, true);
      for (uint32_t i = tid; i < nhot; i += NT) atomicAdd(&dst[S.ev[2 * i]], S.ev[2 * i + 1]);
    } else if (clean && nhot > 0) {
      // ---- hot keys: merge the table into one entry per key holding the
      // bin's total (its field plus all its entries), flag the hot bins, and
      // read counts through the table where flagged ------------------------
      uint32_t tot = 0, live = 0;
      if (tid < nhot) {
        const uint32_t k = S.ev[2 * tid];
        live = 1;
        for (uint32_t j = 0; j < tid; ++j)
          if (S.ev[2 * j] == k) live = 0;  // an earlier entry holds this key
        if (live) {
          tot = packed_count(S, k);
          for (uint32_t j = tid; j < nhot; ++j)
            if (S.ev[2 * j] == k) tot += S.ev[2 * j + 1];
        }
      }
      __syncthreads();
      if (tid < nhot) {
        const uint32_t k = S.ev[2 * tid];
        if (live) {
          S.ev[2 * tid + 1] = tot;
          atomicOr(&S.evflag[k >> 5], 1u << (k & 31));
        }
      }
      __syncthreads();
      if (tid < nhot && !live) S.ev[2 * tid] = 0xFFFFFFFFu;  // no bin matches it
      __syncthreads();
      emit_bins<NT, true, HALIGNED>(S, dst, dhb, 0, cnt, false, nhot);
      if constexpr (FULL) {
        if (gathered)
          project_piece<NT, W / NT, true>(S, status, nitems, items, item_cap, CL2, bp.base, hb, cnt, klast, nhot);
      }
    } else if (clean) {
      // ---- no field wrapped, no hot key -----------------------------------
      emit_bins<NT, true, HALIGNED>(S, dst, dhb, 0, cnt, split);
      if constexpr (FULL) {
        if (!split && gathered)
          project_piece<NT, W / NT, true>(S, status, nitems, items, item_cap, CL2, bp.base, hb, cnt, klast);
      }
    } else {
      // ---- a field wrapped: two halves of 2^15 bins with 32-bit counters ---
      uint64_t hbase = bp.base;  // where the current half's run starts
      for (uint32_t half = 0; half < 2; ++half) {
        const uint32_t hb0 = half << 15;
        if (hb0 >= cnt) break;
        const uint32_t hcnt = cnt - hb0 < (1u << 15) ? cnt - hb0 : (1u << 15);
        __syncthreads();
        for (uint32_t i = tid; i < SM::WORDS; i += NT) S.s[i] = 0;
        __syncthreads();
        bucket_gather<NT, LOG2W, AGG, GM_HALF, TK>(S, staging, seg, bstride, bp.t0, bp.t1, b, half);
        __syncthreads();
        emit_bins<NT, false, HALIGNED>(S, dst, dhb, hb0, hcnt, split);
        if constexpr (FULL) {
          if (!split)
            hbase += project_piece<NT, (1u << 15) / NT, false>(S, status, nitems, items, item_cap, CL2, hbase,
                                                               hb + hb0, hcnt, klast);
        }
      }
    }
  }
  if (!split) return;

  // ---- a part of a heavy bucket: the last part to finish completes it ------
  // every wave waits until its own atomics are acknowledged; then thread 0
  // counts the part as done
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) S.n = __hip_atomic_fetch_add(bp.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (S.n != bp.P - 1) return;
  constexpr uint32_t PW = W < (1u << 15) ? W : (1u << 15);  // bins per piece
  uint64_t pbase = bp.base;
  for (uint32_t p0 = 0; p0 < cnt; p0 += PW) {
    const uint32_t pcnt = cnt - p0 < PW ? cnt - p0 : PW;
    __syncthreads();
    // every part's adds are complete: read them with device-scope loads
    for (uint32_t i = tid; i < PW; i += NT) {
      uint32_t c = 0;
      if (i < pcnt) {
        c = __hip_atomic_load(&bp.acc[p0 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        H[hb + p0 + i] = c;
      }
      S.s[i] = c;
    }
    __syncthreads();
    if constexpr (FULL)
      pbase += project_piece<NT, PW / NT, false>(S, status, nitems, items, item_cap, CL2, pbase, hb + p0, pcnt,
                                                 klast);
  }
}

// The split plan, computed by every workgroup of the bucket pass from the
// partition's bucket-total counters (the same result in each): which part of
// which bucket workgroup `blk` counts, and the run start of that bucket.  A
// bucket is heavy when it holds more than 2 * chunk keys; the SPLIT_SLOTS
// heaviest (among the first HEAVY_MAX heavy buckets in bucket order) get
// scratch slots and want ceil(total / chunk) - 1 extra parts each, handed out
// heaviest first while the X extra workgroups last.  Workgroup i < B takes part 0 of a bucket
// (XCD-aware order: blocks are dispatched round-robin over 8 XCDs, so each XCD
// takes a contiguous range of buckets); workgroup B + e takes extra part e, if
// it exists.  Returns false for a workgroup without a part.
template <int NT, typename SM>
__device__ __forceinline__ bool plan_part(SM& S, const SplitPlan& plan, uint32_t B, uint32_t T, uint32_t blk,
                                          BucketPart& bp) {
  static_assert(SM::WORDS >= PART_BMAX + 3 * SPLIT_SLOTS + HEAVY_MAX, "totals and tables fit the counters");
  static_assert(HEAVY_MAX <= NT, "one thread per listed heavy bucket");
  uint32_t* tot = S.s;               // per bucket
  uint32_t* tab = S.s + PART_BMAX;   // per slot: bucket, first extra part, extra parts wanted
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < B; i += NT) tot[i] = 0;
  __syncthreads();
  const uint32_t ncnt = plan.rows * B;
#pragma unroll 4
  for (uint32_t i = tid; i < ncnt; i += NT) {
    const uint32_t v = plan.colsum[i];
    if (v) atomicAdd(&tot[i % B], v);
  }
  __syncthreads();
  // heavy buckets, listed in bucket order (at most HEAVY_MAX of them), then
  // ranked by total, heaviest first (ties: lower bucket first)
  uint32_t* hl = tab + 3 * SPLIT_SLOTS;  // heavy list: bucket indices
  uint32_t nheavy = 0;
  for (uint32_t r0 = 0; r0 < B; r0 += NT) {
    const uint32_t bb = r0 + tid;
    const uint32_t heavy = plan.X > 0 && bb < B && (uint64_t)tot[bb] > 2 * plan.chunk ? 1u : 0u;
    uint32_t round_heavy;
    const uint32_t at = nheavy + block_exclusive_sum<NT>(heavy, reinterpret_cast<uint32_t*>(S.red), &round_heavy);
    if (heavy && at < HEAVY_MAX) hl[at] = bb;
    nheavy += round_heavy;
  }
  if (nheavy > HEAVY_MAX) nheavy = HEAVY_MAX;
  __syncthreads();
  if (tid < nheavy) {
    const uint32_t mb = hl[tid];
    const uint32_t mt = tot[mb];
    uint32_t rank = 0;
    for (uint32_t j = 0; j < nheavy; ++j) {
      const uint32_t ob = hl[j], ot = tot[ob];
      rank += (ot > mt || (ot == mt && ob < mb)) ? 1u : 0u;
    }
    if (rank < SPLIT_SLOTS) {
      tab[3 * rank] = mb;
      const uint64_t w = ((uint64_t)mt + plan.chunk - 1) / plan.chunk - 1;
      tab[3 * rank + 2] = w < plan.X ? (uint32_t)w : plan.X;
    }
  }
  __syncthreads();
  const uint32_t nslot = nheavy < SPLIT_SLOTS ? nheavy : SPLIT_SLOTS;
  if (tid == 0) {
    uint32_t first = 0;  // extra parts go to the slots in rank order
    for (uint32_t sl = 0; sl < nslot; ++sl) {
      tab[3 * sl + 1] = first;
      first += tab[3 * sl + 2];
    }
  }
  __syncthreads();
  // extra parts a slot got: its wants, cut at X
  auto got = [&](uint32_t sl) -> uint32_t {
    const uint32_t first = tab[3 * sl + 1], want = tab[3 * sl + 2];
    return first >= plan.X ? 0u : (want < plan.X - first ? want : plan.X - first);
  };
  uint32_t b = 0, p = 0;
  if (blk < B) {
    b = blk;
    if ((B & 7u) == 0) b = (blk & 7u) * (B >> 3) + (blk >> 3);
  } else {
    const uint32_t e = blk - B;
    bool found = false;
    for (uint32_t sl = 0; sl < nslot; ++sl) {
      const uint32_t first = tab[3 * sl + 1];
      if (e >= first && e < first + got(sl)) {
        b = tab[3 * sl];
        p = 1 + (e - first);
        found = true;
      }
    }
    if (!found) return false;  // the same in every thread
  }
  bp.b = b;
  bp.P = 1;
  bp.acc = nullptr;
  bp.done = nullptr;
  for (uint32_t sl = 0; sl < nslot; ++sl) {
    if (tab[3 * sl] == b && got(sl) > 0) {
      bp.P = 1 + got(sl);
      bp.acc = plan.scratch + (uint64_t)sl * PART_W;
      bp.done = plan.done + sl;
    }
  }
  bp.t0 = (uint32_t)((uint64_t)p * T / bp.P);
  bp.t1 = (uint32_t)((uint64_t)(p + 1) * T / bp.P);
  uint64_t below = 0;
  for (uint32_t bb = tid; bb < b; bb += NT) below += tot[bb];
  bp.base = block_sum<NT>(S, below);  // ends with a barrier: S.s is free again
  return true;
}

template <int AGG, bool HALIGNED, bool FULL>
__global__ __launch_bounds__(PART_NT) void k_bucket(const uint16_t* __restrict__ staging,
                                                    const uint16_t* __restrict__ seg, uint32_t bstride,
                                                    uint32_t T, uint32_t B, uint64_t U, uint32_t* __restrict__ H,
                                                    Ctl* ctl, FillItem* __restrict__ items, uint32_t item_cap,
                                                    int CL2, SplitPlan plan) {
  __shared__ __align__(16) BinSmem<PART_NT, PART_LOG2W> S;
  BucketPart bp;
  if (!plan_part<PART_NT>(S, plan, B, T, blockIdx.x, bp)) return;
  bucket_body<PART_NT, PART_LOG2W, AGG, HALIGNED, FULL, PART_TK>(S, staging, seg, bstride, U, H, &ctl->status,
                                                                &ctl->nitems, items, item_cap, CL2, bp);
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
