// Ordered projection (DialSort Sec. 3.3, Eq. (2)): emit k exactly H[k] times for
// k = 0 .. U-1.
//
// The paper's sequential projection keeps one output cursor.  In parallel every
// bin needs its starting position, the exclusive prefix of H; the paper does not
// say how its 8-thread version splits the scan, so the split here is ours:
//
// k_scan: one pass over H with a single-pass decoupled look-back (tile t
//   publishes its aggregate, then adds its predecessors' aggregates until it
//   meets an inclusive prefix; tiles are numbered by a ticket taken at start, so
//   every tile waits only on tiles that are already running).  The same pass can
//   first sum the partial-histogram rows written by the LDS ingestion kernels
//   and store the result as H.  Each tile then cuts its output span at the
//   multiples of C and appends one fill item per piece: (first position, end,
//   first bin, that bin's run start, end bin).  An item therefore covers at most
//   C positions and at most one tile of bins, whatever the skew (a hot key of
//   10^8 copies becomes 10^8 / C items) and however sparse H is.
//
// k_fill: persistent waves take items, each wave on its own.  An item walks
//   its bins, marks the position where each run begins, and fills its
//   positions by carrying every marked key forward to the next mark; interior
//   stores are 16-byte coalesced stores.  Zero bins emit nothing (the presence test of Sec. 2, Table
//   "tab:comparison", is not an order comparison).
#pragma once

#include "common.hpp"
#include "fill_window.hpp"

namespace ds {

constexpr uint64_t LB_FLAG_A = 1ull << 62;  // aggregate available
constexpr uint64_t LB_FLAG_P = 2ull << 62;  // inclusive prefix available
constexpr uint64_t LB_VAL = (1ull << 62) - 1;

// One piece of the projection: output positions [p0, p1) (p1 - p0 <= C, and
// [p0 & ~3, p1) fits in C), whose first position is covered by bin k with run
// start o <= p0; the bins to walk are k .. klast (the end of k's scan tile).
struct FillItem {
  uint64_t p0, p1, o;
  uint32_t k, klast;
};
static_assert(sizeof(FillItem) == 32, "fill items are 32 bytes");

// A long run of the scan: bin k's run [o, o + H[k]) holds more than RUN_MIN
// chunk starts; its items (chunks c0 .. c0 + cnt - 1, each [c C, min((c+1) C,
// e0)), walking bins k .. klast) are not stored but made by the fill from this
// record.  Runs are numbered in the order they take their chunks, so `start`
// (the number of run chunks before this run's first) grows with the index.
struct FillRun {
  uint64_t start, c0, o, e0;
  uint32_t k, klast;
};
static_assert(sizeof(FillRun) == 40, "run records are 40 bytes");
constexpr uint64_t RUN_MIN = 4;              // a run with more chunk starts is recorded, not expanded
constexpr int RUN_SHIFT = 40;                // Ctl::runs = (runs << RUN_SHIFT) | chunks
constexpr uint64_t RUN_CHUNKS = (1ull << RUN_SHIFT) - 1;

// The fill item of run chunk j (0 <= j < total run chunks) among `nruns` runs.
__device__ __forceinline__ FillItem run_item(const FillRun* __restrict__ runs, uint32_t nruns, uint64_t j, int CL2) {
  uint32_t lo = 0, hi = nruns;  // the last run with start <= j
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (runs[mid].start <= j) lo = mid; else hi = mid;
  }
  const FillRun R = runs[lo];
  const uint64_t c = R.c0 + (j - R.start);
  FillItem it;
  it.p0 = c << CL2;
  it.p1 = ((c + 1) << CL2) < R.e0 ? ((c + 1) << CL2) : R.e0;
  it.o = R.o;
  it.k = R.k;
  it.klast = R.klast;
  return it;
}

__device__ __forceinline__ uint64_t wave_sum_sat(uint64_t x) {
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) x = sat_add(x, __shfl_xor(x, d, WAVE));
  return x;
}

// Decoupled look-back for tile t (called by wave 0 of the block).  Returns the
// exclusive prefix of tile t (all lanes get it).  A round reads LB_GROUPS x 64
// predecessors at once (lane l of group i reads tile j - 64 i - l), so a tile
// far from the last published prefix reaches it in few round trips.  Groups
// are taken nearest first; a group with an unpublished tile before its first
// prefix is read again, from that group on, in the next round.
constexpr int LB_GROUPS = 4;
__device__ __forceinline__ uint64_t lookback(uint64_t* state, uint64_t t) {
  const int lane = lane_id();
  uint64_t prefix = 0;
  int64_t j = (int64_t)t - 1;  // the nearest predecessor not yet added
  for (;;) {
    uint64_t s[LB_GROUPS];
#pragma unroll
    for (int i = 0; i < LB_GROUPS; ++i) {
      const int64_t idx = j - i * WAVE - lane;
      s[i] = idx >= 0 ? ld_acquire_u64(&state[idx]) : LB_FLAG_P;
    }
    bool pending = false;
#pragma unroll
    for (int i = 0; i < LB_GROUPS; ++i) {
      const uint64_t pm = __ballot((s[i] >> 62) == 2);
      const int p = pm ? __ffsll((unsigned long long)pm) - 1 : WAVE - 1;  // the lanes this group needs: 0 .. p
      if (__ballot((s[i] >> 62) == 0) & ((2ull << p) - 1)) { pending = true; break; }
      prefix = sat_add(prefix, wave_sum_sat(lane <= p ? (s[i] & LB_VAL) : 0));
      if (pm) return prefix;
      j -= WAVE;
    }
    if (pending) __builtin_amdgcn_s_sleep(1);
  }
}

// NT threads, VPT bins per thread (tile = NT*VPT bins).
// rows: nrows partial rows (row r at rows + r*row_stride); H_out receives their
// sum when non-null.  FULL: also scan and build the chunk map (chunk = 2^CL2).
// DIRECT (with FULL): instead of fill items, every tile writes its own runs
// into out once its prefix is known (wave_fill; the counts must come from keys,
// so that any sum of them fits 32 bits).
// limit: number of output positions that may be written (n, or out_cap).
// row16: the rows hold 16-bit counts (bin k is halfword k of its row).
template <int NT, int VPT, bool FULL, bool DIRECT = false>
__global__ __launch_bounds__(NT) void k_scan(const uint32_t* __restrict__ rows, uint32_t nrows, uint64_t row_stride,
                                             uint32_t* __restrict__ H_out, uint64_t U, Ctl* ctl,
                                             uint64_t* tile_state, FillItem* __restrict__ items,
                                             uint32_t item_cap, uint64_t limit, int CL2, int report_overflow,
                                             FillRun* __restrict__ runs, uint32_t run_cap, uint32_t* __restrict__ out,
                                             FillCfg fc, uint32_t row_status, uint32_t row16) {
  constexpr int TB = NT * VPT;
  constexpr int PADW = TB + TB / 32;
  __shared__ uint32_t tr[VPT > 1 ? PADW : 1];
  __shared__ __align__(16) uint32_t wbuf[DIRECT ? NT / WAVE : 1][DIRECT ? WIN_POS : 1];
  __shared__ uint64_t scan_tmp[NT / WAVE + 1];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_item0;
  const uint32_t tid = threadIdx.x;

  // row_status: each partial row holds its ingestion's status bits in word U
  if (row_status && blockIdx.x == 0) {
    uint32_t bits = 0;
    for (uint32_t r = tid; r < nrows; r += NT) bits |= rows[(uint64_t)r * row_stride + U];
    if (bits) atomicOr(&ctl->status, bits);  // only on a faulty input
  }

  uint64_t t = blockIdx.x;
  if constexpr (FULL) {
    if (tid == 0) s_tile = atomicAdd(&ctl->tile_ticket, 1u);
    __syncthreads();
    t = s_tile;
  }
  const uint64_t base = t * (uint64_t)TB;

  // 1. sum the rows (striped layout: bin base + j*NT + tid)
  uint32_t v[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const uint64_t k = base + (uint64_t)j * NT + tid;
    uint32_t a = 0;
    if (k < U) {
      const uint16_t* rows16 = reinterpret_cast<const uint16_t*>(rows);
      if constexpr (VPT == 1) {
        // one bin per thread: 32 (16-bit rows) or 16 rows' loads in flight at once
        if (row16) {
#pragma unroll 32
          for (uint32_t r = 0; r < nrows; ++r) a += rows16[(uint64_t)r * row_stride * 2 + k];
        } else {
#pragma unroll 16
          for (uint32_t r = 0; r < nrows; ++r) a += rows[(uint64_t)r * row_stride + k];
        }
      } else {
        if (row16) {
#pragma unroll 8
          for (uint32_t r = 0; r < nrows; ++r) a += rows16[(uint64_t)r * row_stride * 2 + k];
        } else {
#pragma unroll 8
          for (uint32_t r = 0; r < nrows; ++r) a += rows[(uint64_t)r * row_stride + k];
        }
      }
      if (H_out) H_out[k] = a;
    }
    v[j] = a;
  }
  if constexpr (!FULL) return;

  // 2. blocked layout: thread tid owns bins base + tid*VPT .. + VPT-1
  if constexpr (VPT > 1) {
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const uint32_t p = j * NT + tid;
      tr[p + (p >> 5)] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const uint32_t p = tid * VPT + j;
      v[j] = tr[p + (p >> 5)];
    }
  }
  uint64_t tsum = 0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) tsum += v[j];
  uint64_t agg;
  const uint64_t texcl = block_exclusive_sum<NT>(tsum, scan_tmp, &agg);
  const uint64_t agg_sat = agg > LB_VAL ? LB_VAL : agg;

  // 3. decoupled look-back across tiles
  if (tid < WAVE) {
    if (t == 0) {
      if (tid == 0) { st_release_u64(&tile_state[0], LB_FLAG_P | agg_sat); s_prefix = 0; }
    } else {
      if (tid == 0) st_release_u64(&tile_state[t], LB_FLAG_A | agg_sat);
      const uint64_t pre = lookback(tile_state, t);
      if (tid == 0) {
        st_release_u64(&tile_state[t], LB_FLAG_P | sat_add(pre, agg_sat));
        s_prefix = pre;
      }
    }
  }
  __syncthreads();
  const uint64_t tpre = s_prefix;
  const uint64_t ntiles = (U + TB - 1) / TB;
  if (t == ntiles - 1 && tid == 0) {
    const uint64_t total = sat_add(tpre, agg_sat);
    const uint64_t lim = total < limit ? total : limit;
    ctl->total = total;
    ctl->limit = lim;
    if (report_overflow && total > limit) set_status(ctl, ST_OVERFLOW);
  }

  if constexpr (DIRECT) {
    // 4'. the tile's runs, written by its waves: wave w owns the tile's bins
    //     [64 VPT w, 64 VPT (w + 1)), whose run starts where its lane 0's
    //     stretch starts (blocked layout)
    const uint32_t lane = lane_id(), w = tid / WAVE;
    const uint64_t wstart = sat_add(tpre, (uint64_t)__shfl((long long)texcl, 0, WAVE));
    const uint64_t wtot = wave_sum(tsum);
    auto count = [&](uint32_t j) -> uint32_t {
      if constexpr (VPT == 1) {
        return v[0];
      } else {
        const uint32_t p = w * (WAVE * VPT) + j * WAVE + lane;  // bin - base
        return tr[p + (p >> 5)];
      }
    };
    wave_fill(wbuf[w], out, wstart, wtot, base + (uint64_t)w * WAVE * VPT, VPT, count, fc);
    return;
  }

  // 4. fill items of this tile: its span [s, e), clipped at limit, cut at the
  //    multiples of C.  Item 0 starts at s; item j >= 1 at (floor(s/C) + j) * C.
  const uint64_t C = 1ull << CL2;
  const uint64_t s0 = tpre < limit ? tpre : limit;
  const uint64_t e0 = sat_add(tpre, agg_sat) < limit ? sat_add(tpre, agg_sat) : limit;
  const uint64_t cbase = s0 >> CL2;
  const uint64_t nit = e0 > s0 ? ((e0 + C - 1) >> CL2) - cbase : 0;
  // chunk starts c*C strictly inside the span and inside bin's run [o, o+h)
  auto starts = [&](uint64_t o, uint64_t h, uint64_t& c0, uint64_t& cnt) {
    c0 = 0; cnt = 0;
    if (nit > 0 && h > 0 && o < e0) {
      const uint64_t e = sat_add(o, h) < e0 ? sat_add(o, h) : e0;  // run clipped to the span
      uint64_t lo = (o + C - 1) >> CL2;
      if (lo < cbase + 1) lo = cbase + 1;
      const uint64_t hi = (e - 1) >> CL2;
      c0 = lo;
      cnt = hi >= lo ? hi - lo + 1 : 0;
    }
  };
  // Runs with more than RUN_MIN chunk starts become run records; the other
  // chunks are stored as items, numbered in position order without the run
  // chunks (a block scan counts the run chunks before each thread's bins).
  const uint64_t o_first = sat_add(tpre, texcl);
  uint64_t my_lr = 0;
  {
    uint64_t o = o_first;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      uint64_t c0, cnt;
      starts(o, v[j], c0, cnt);
      if (cnt > RUN_MIN) my_lr += cnt;
      o = sat_add(o, v[j]);
    }
  }
  uint64_t lr_total = 0, lr_seen = 0;
  if (__syncthreads_or(my_lr != 0)) lr_seen = block_exclusive_sum<NT>(my_lr, scan_tmp, &lr_total);
  if (tid == 0) {
    uint32_t i0 = 0;
    const uint64_t nreg = nit - lr_total;
    if (nreg) {
      i0 = atomicAdd(&ctl->nitems, (uint32_t)nreg);
      if ((uint64_t)i0 + nreg > item_cap) { set_status(ctl, ST_INT_ITEMS); i0 = 0xFFFFFFFFu; }
    }
    s_item0 = i0;
  }
  __syncthreads();
  const uint32_t item0 = s_item0;
  const bool emit = nit > 0 && item0 != 0xFFFFFFFFu;
  const uint32_t klast = (uint32_t)((base + TB < U ? base + TB : U) - 1);
  uint64_t o = o_first;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const uint64_t h = v[j];
    const uint64_t bin = base + (uint64_t)tid * VPT + j;
    uint64_t c0, cnt;
    starts(o, h, c0, cnt);
    if (emit && h > 0 && o < e0 && o == s0) {  // the first nonzero bin opens item 0
      FillItem it;
      it.p0 = s0; it.p1 = ((cbase + 1) << CL2) < e0 ? ((cbase + 1) << CL2) : e0;
      it.o = o; it.k = (uint32_t)bin; it.klast = klast;
      items[item0] = it;
    }
    if (emit && cnt > 0 && cnt <= RUN_MIN) {
      for (uint64_t i = 0; i < cnt; ++i) {
        const uint64_t c = c0 + i;
        FillItem it;
        it.p0 = c << CL2; it.p1 = ((c + 1) << CL2) < e0 ? ((c + 1) << CL2) : e0;
        it.o = o; it.k = (uint32_t)bin; it.klast = klast;
        items[item0 + (c - cbase) - lr_seen] = it;
      }
    }
    if (emit && cnt > RUN_MIN) {
      const uint64_t old = atomicAdd((unsigned long long*)&ctl->runs, (1ull << RUN_SHIFT) | cnt);
      const uint64_t slot = old >> RUN_SHIFT;
      if (slot < run_cap) {
        FillRun r;
        r.start = old & RUN_CHUNKS; r.c0 = c0; r.o = o; r.e0 = e0; r.k = (uint32_t)bin; r.klast = klast;
        runs[slot] = r;
      } else {
        set_status(ctl, ST_INT_ITEMS);
      }
      lr_seen += cnt;
    }
    o = sat_add(o, h);
  }
}

// Fill of one item by ONE wavefront, with no workgroup barrier: every wave of
// a workgroup takes its own items.  C = 2^CL2 local positions per item (C/32
// <= 64 flag words, one per lane).  Local position i is output position a0 + i
// with a0 = p0 rounded down to a multiple of 4; an item always fits in [0, C)
// of that frame.  The wave's LDS: val[0, C) holds the key marked at each run
// start, val[C + s] the key carried into 32-position segment s (the last mark
// before it), flag[s] the marks of segment s.  Keys are kept as 16-bit offsets
// from the item's first bin (an item spans at most FILL_SPAN_MAX bins), which
// halves the wave's LDS and doubles the waves a CU holds.  LDS operations of
// one wave take effect in program order, so no fence is needed between the
// phases.
constexpr uint32_t FILL_SPAN_MAX = 65536;  // bins of one fill item (klast - k < this)

template <int CL2>
struct WaveFillSmem {
  static constexpr uint32_t C = 1u << CL2;
  static constexpr uint32_t NFW = C / 32;
  __align__(16) uint16_t val[C + NFW];
  uint32_t flag[NFW];
};

// LUT: bin k's value is lut[k] (a table phi^-1 of Sec. 3.4) instead of lo + k.
// NTS: the 16-byte stores are non-temporal (streamed past the caches).
template <int CL2, bool OALIGNED, bool LUT = false, bool NTS = false>
__device__ __forceinline__ void wave_fill_item(WaveFillSmem<CL2>& S, const uint32_t* __restrict__ H,
                                               uint32_t* __restrict__ out, const FillItem& I, uint32_t lo = 0,
                                               const uint32_t* __restrict__ lut = nullptr) {
  constexpr uint32_t C = 1u << CL2;
  constexpr uint32_t NFW = C / 32;
  static_assert(NFW <= (uint32_t)WAVE, "one flag word per lane at most");
  const uint32_t lane = lane_id();
  // output quads q = lane + 64 r all sit at the same offset b0 = 4 (q mod 8)
  // inside their 32-position segment: the masks of positions <= b0 + e are fixed
  const uint32_t b0 = (lane & 7u) * 4u;
  const uint32_t mk0 = 0xFFFFFFFFu >> (31u - b0), mk1 = 0xFFFFFFFFu >> (30u - b0);
  const uint32_t mk2 = 0xFFFFFFFFu >> (29u - b0), mk3 = 0xFFFFFFFFu >> (28u - b0);

  const uint64_t p0 = I.p0, p1 = I.p1;
  const uint64_t a0 = p0 & ~3ull;
  const uint32_t lb = (uint32_t)(p0 - a0), le = (uint32_t)(p1 - a0);  // local [lb, le) within [0, C)
  if (lane < NFW) S.flag[lane] = 0;
  // walk the item's bins, 4 per lane per round, marking run starts in [p0, p1)
  uint64_t kb = I.k;
  uint64_t run = I.o;  // start position of bin kb's run (<= p0)
  while (run < p1 && kb <= I.klast) {  // wave-uniform
    const uint64_t k0 = kb + 4ull * lane;
    uint32_t h[4];
    uint64_t tsum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      h[j] = k0 + j <= I.klast ? H[k0 + j] : 0u;
      tsum += h[j];
    }
    const uint64_t inc = wave_inclusive_sum(tsum);
    const uint64_t tot = __shfl(inc, WAVE - 1, WAVE);
    uint64_t ok = run + inc - tsum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (h[j] > 0 && ok < p1) {
        const uint32_t pos = ok <= p0 ? lb : (uint32_t)(ok - a0);
        S.val[pos] = (uint16_t)(k0 + j - I.k);
        atomicOr(&S.flag[pos >> 5], 1u << (pos & 31));
      }
      ok += h[j];
    }
    run += tot;
    kb += 4ull * WAVE;
  }
  // carry the last mark forward: lane s owns segment s; segment 0 always holds
  // the item's first mark (at lb <= 3)
  const uint32_t f = lane < NFW ? S.flag[lane] : 0u;
  int32_t inc = f ? (int32_t)lane : -1;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int32_t y = __shfl_up(inc, d, WAVE);
    if ((int)lane >= d && y > inc) inc = y;
  }
  int32_t ex_idx = __shfl_up(inc, 1, WAVE);
  if (lane == 0) ex_idx = -1;
  if (lane < NFW) {
    uint32_t cin = 0;
    if (ex_idx >= 0) cin = S.val[ex_idx * 32 + (31 - __clz(S.flag[ex_idx]))];
    S.val[C + lane] = cin;
  }
  // every output quad resolves its keys from its segment's flag word: the key
  // at position p is the last mark at or before p in the segment, else the
  // segment's carried key
  const uint32_t nq = (le + 3) >> 2;
  // phi^-1 (Sec. 3.4): bin k holds key lo + k, or lut[k]
  const uint32_t kf = LUT ? I.k : I.k + lo;
  const uint32_t* __restrict__ tab = LUT ? lut + I.k : nullptr;
  for (uint32_t q = lane; q < nq; q += WAVE) {
    const uint32_t sg = q >> 3;
    const uint32_t fw = S.flag[sg];
    uint32_t r0, r1, r2, r3;
    if (fw == 0) {
      r0 = r1 = r2 = r3 = LUT ? tab[S.val[C + sg]] : kf + S.val[C + sg];
    } else {
      const uint32_t base = sg * 32u + 31u;
      const uint32_t m0 = fw & mk0, m1 = fw & mk1, m2 = fw & mk2, m3 = fw & mk3;
      const uint32_t o0 = S.val[m0 ? base - __clz(m0) : C + sg], o1 = S.val[m1 ? base - __clz(m1) : C + sg];
      const uint32_t o2 = S.val[m2 ? base - __clz(m2) : C + sg], o3 = S.val[m3 ? base - __clz(m3) : C + sg];
      if (LUT) {
        r0 = tab[o0];
        r1 = tab[o1];
        r2 = tab[o2];
        r3 = tab[o3];
      } else {
        r0 = kf + o0;
        r1 = kf + o1;
        r2 = kf + o2;
        r3 = kf + o3;
      }
    }
    const uint32_t i0 = q << 2;
    if (OALIGNED && i0 >= lb && i0 + 4 <= le) {
      if constexpr (NTS) {
        typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
        const u32x4_t v = {r0, r1, r2, r3};
        __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t*>(out + a0 + i0));
      } else {
        *reinterpret_cast<uint4*>(out + a0 + i0) = make_uint4(r0, r1, r2, r3);
      }
    } else {
      if (i0 >= lb && i0 < le) out[a0 + i0] = r0;
      if (i0 + 1 >= lb && i0 + 1 < le) out[a0 + i0 + 1] = r1;
      if (i0 + 2 >= lb && i0 + 2 < le) out[a0 + i0 + 2] = r2;
      if (i0 + 3 >= lb && i0 + 3 < le) out[a0 + i0 + 3] = r3;
    }
  }
}

// Persistent fill over the items appended to ctl->nitems: every wave of every
// workgroup takes items on its own.
template <int NT, int CL2, bool OALIGNED, bool LUT = false, bool NTS = false>
__global__ __launch_bounds__(NT) void k_fill(const uint32_t* __restrict__ H, uint32_t* __restrict__ out,
                                             Ctl* ctl, const FillItem* __restrict__ items,
                                             uint32_t item_cap, uint32_t lo, const uint32_t* __restrict__ lut,
                                             const FillRun* __restrict__ runs, uint32_t run_cap) {
  constexpr uint32_t NW = NT / WAVE;
  __shared__ WaveFillSmem<CL2> S[NW];
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  // a failed invariant (reported as ST_INTERNAL) leaves items unwritten: fill nothing
  const bool failed = (ctl->status & ST_INTERNAL) != 0;
  const uint32_t nitems = failed ? 0u : (ctl->nitems < item_cap ? ctl->nitems : item_cap);
  // the stored items, then the chunks of the recorded runs
  const uint64_t rr = failed ? 0ull : ctl->runs;
  const uint32_t nruns = (uint32_t)(rr >> RUN_SHIFT) < run_cap ? (uint32_t)(rr >> RUN_SHIFT) : run_cap;
  const uint64_t ntotal = nitems + (nruns ? (rr & RUN_CHUNKS) : 0ull);
  const uint64_t stride = (uint64_t)gridDim.x * NW;
  uint64_t it = blockIdx.x * NW + w;
  // the wave's next stored item is loaded while the current one is filled
  FillItem next{};
  if (it < nitems) next = items[it];
  for (; it < ntotal; it += stride) {
    const FillItem I = it < nitems ? next : run_item(runs, nruns, it - nitems, CL2);
    if (it + stride < nitems) next = items[it + stride];
    // every producer cuts items well inside the 16-bit key offsets; anything
    // else is a broken invariant, reported instead of written
    if (I.klast < I.k || I.klast - I.k >= FILL_SPAN_MAX || I.p1 < I.p0 || I.p1 - (I.p0 & ~3ull) > (1ull << CL2)) {
      if (lane_id() == 0) atomicOr(&ctl->status, ST_INT_ITEM);
      continue;
    }
    wave_fill_item<CL2, OALIGNED, LUT, NTS>(S[w], H, out, I, lo, lut);
  }
}

}  // namespace ds
