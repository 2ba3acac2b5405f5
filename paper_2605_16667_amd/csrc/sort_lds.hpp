// A sort of a small input in one launch: Eq. (1) into LDS-privatized partial
// rows, then Eq. (2) projected by slices of bins (DialSort Sec. 3.3).  What one
// launch saves is a second launch, its start-up, and the look-back between
// scan tiles: at 2^20 keys, together with 16-bit rows, a third of the sort.
//
// Blocks [0, G) count slab g of the keys into LDS exactly as k_hist_lds does
// and write partial row g as 16-bit counts (a slab holds fewer than 2^16
// keys).  While writing it, a block also sums its counts per slice of 256 bins
// and stores the exclusive prefix of those sums over the slices (plus the
// slab's total) as pre[g]: the start of slice s in the output is then
// sum_g pre[g][s], with no scan across slices.  Blocks [G, G + NS) each own
// slice s = block - G: once every counting block has published, a block sums
// the G rows over its 256 bins, writes that part of H, and writes the slice's
// runs into the output, 16 bins per wave.
//
// The wait needs no counter that something must clear first: counting block g
// stores the launch's epoch into flag g after its row, and a block goes on once
// all G flags hold it.  The host draws a fresh epoch for every launch from a
// process-wide 64-bit sequence that starts at a random value, so flags left by
// earlier launches (or whatever the workspace held before) do not match.  A
// replayed graph would repeat the epoch, so the host uses this form only on a
// stream that is not capturing.
//
// Progress: counting blocks never wait, and every block that waits has a
// larger index than all of them: blocks are dispatched in index order, so
// whenever a slice block is resident every counting block has been dispatched
// and will finish, whatever else shares the device (other launches of this
// kernel included).  The wait is bounded all the same: after FUSED_WAIT_TICKS
// of the 100 MHz clock a block stops waiting and reports ST_INT_WAIT.
//
// Publication across XCDs: a counting block waits until its stores are
// acknowledged, passes a barrier, and thread 0 stores the flag with release
// semantics at agent scope (which writes this XCD's L2 back first); a waiting
// block polls with relaxed loads and then fences with acquire semantics at
// agent scope before any of its threads reads a row.
#pragma once

#include "common.hpp"
#include "fill_window.hpp"
#include "hist_lds.hpp"

namespace ds {

constexpr uint64_t FUSED_WAIT_TICKS = 200000000ull;  // 2 s
constexpr uint32_t SLICE = SLICE_BINS;
constexpr uint32_t FUSED_SLICES_MAX = 256;

template <int NT>
struct SliceSmem {
  static constexpr uint32_t RG = NT / (SLICE / 2);  // row groups: thread t reads word t mod 128 of rows = t / 128 (mod RG)
  uint2 part[RG][SLICE / 2];
  uint32_t cnt[SLICE];
  uint32_t excl[SLICE + 1];
  uint32_t pre[NT / WAVE], tot[NT / WAVE], wsum[NT / WAVE];
  __align__(16) uint32_t wbuf[NT / WAVE][WIN_POS];
};

template <int NT, int CAP, bool PACKED, int AGG, bool ALIGNED, int UNR>
__global__ __launch_bounds__(NT) void k_sort_lds(const uint32_t* __restrict__ keys, uint64_t n, uint64_t per,
                                                 uint32_t umax, uint32_t U, uint32_t G, uint32_t NS,
                                                 uint32_t* __restrict__ rows, uint64_t row_stride,
                                                 uint32_t* __restrict__ pre, Ctl* ctl, uint64_t* flags, uint64_t epoch,
                                                 uint32_t* __restrict__ H, uint32_t* __restrict__ out, FillCfg fc) {
  static_assert(NT == 16 * WAVE, "16 waves of 16 bins cover a slice");
  __shared__ union {
    HistSmem<CAP, PACKED> h;
    SliceSmem<NT> s;
  } S;
  __shared__ uint32_t scnt[FUSED_SLICES_MAX];
  const uint32_t b = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  const uint64_t P1 = (uint64_t)NS + 1;  // entries of pre per slab

  if (b < G) {
    // counting block: as k_hist_lds with the clearing folded in (block 0
    // clears the control block; nothing else of it is used before the wait)
    if (b == 0 && tid < sizeof(Ctl) / 4) reinterpret_cast<uint32_t*>(ctl)[tid] = 0;
    for (uint32_t i = tid; i < NS; i += NT) scnt[i] = 0;  // hist_slab's first barrier orders this before use
    const uint64_t beg = (uint64_t)b * per;
    const uint64_t end = beg + per < n ? beg + per : n;
    uint32_t* row = rows + (uint64_t)b * row_stride;
    uint32_t* status = row + U;
    if (tid == 0) *status = 0;
    hist_slab<NT, PACKED, AGG, ALIGNED, UNR>(S.h, keys, beg, end, umax, U, row, status, fc.lo, true, scnt);
    __syncthreads();
    if (tid < WAVE) {
      uint32_t carry = 0;
      for (uint32_t s0 = 0; s0 < NS; s0 += WAVE) {
        const uint32_t s = s0 + lane;
        const uint32_t c = s < NS ? scnt[s] : 0u;
        const uint32_t inc = wave_inclusive_sum(c);
        if (s < NS) pre[(uint64_t)b * P1 + s] = carry + inc - c;
        carry += (uint32_t)__shfl((int)inc, WAVE - 1, WAVE);
      }
      if (lane == 0) pre[(uint64_t)b * P1 + NS] = carry;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&flags[b], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const uint32_t sl = b - G;  // this block's slice

  if (tid < WAVE) {
    const uint64_t t0 = wall_clock64();
    bool late = false;
    for (;;) {
      bool mine = true;
      for (uint32_t g = lane; g < G; g += WAVE)
        mine &= __hip_atomic_load(&flags[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
      if (__all(mine)) break;
      if (wall_clock64() - t0 > FUSED_WAIT_TICKS) { late = true; break; }
      __builtin_amdgcn_s_sleep(2);
    }
    if (late && lane == 0) set_status(ctl, ST_INT_WAIT);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();

  // each row's status word (a key past U in its slab) into the control block
  if (sl == 0) {
    uint32_t bits = 0;
    for (uint32_t g = tid; g < G; g += NT) bits |= rows[(uint64_t)g * row_stride + U];
    if (bits) atomicOr(&ctl->status, bits);
  }

  // 1. the slice's counts: thread t sums word t mod 128 of the slice (bins
  //    2w, 2w + 1) over rows t / 128, + RG, ...; the slice's start and (last
  //    slice) the total from pre
  const uint64_t sbase = (uint64_t)sl << SLICE_LOG2;
  {
    constexpr uint32_t RG = SliceSmem<NT>::RG;
    const uint32_t w = tid % (SLICE / 2), h = tid / (SLICE / 2);
    uint32_t lo16 = 0, hi16 = 0;
    if (sbase + 2 * w < U) {
      const uint32_t* rw = rows + (sbase >> 1) + w;
#pragma unroll 8
      for (uint32_t r = h; r < G; r += RG) {
        const uint32_t x = rw[(uint64_t)r * row_stride];
        lo16 += x & 0xFFFFu;
        hi16 += x >> 16;
      }
    }
    S.s.part[h][w] = make_uint2(lo16, hi16);
    uint32_t pg = 0, tg = 0;
    if (tid < G) {
      pg = pre[(uint64_t)tid * P1 + sl];
      if (sl == NS - 1) tg = pre[(uint64_t)tid * P1 + NS];
    }
    pg = wave_sum(pg);
    tg = wave_sum(tg);
    if (lane == 0) { S.s.pre[wv] = pg; S.s.tot[wv] = tg; }
  }
  __syncthreads();
  uint32_t c = 0;
  if (tid < SLICE) {
#pragma unroll
    for (uint32_t h = 0; h < SliceSmem<NT>::RG; ++h) {
      const uint2 p = S.s.part[h][tid >> 1];
      c += (tid & 1u) ? p.y : p.x;
    }
    if (sbase + tid < U) H[sbase + tid] = c;
    const uint32_t inc = wave_inclusive_sum(c);
    S.s.cnt[tid] = c;
    S.s.excl[tid] = inc - c;  // within the wave for now
    if (lane == WAVE - 1) S.s.wsum[wv] = inc;
  }
  __syncthreads();
  uint64_t spre = 0;
#pragma unroll
  for (uint32_t i = 0; i < NT / WAVE; ++i) spre += S.s.pre[i];
  if (tid < SLICE) {
    uint32_t before = 0;
    for (uint32_t i = 0; i < wv; ++i) before += S.s.wsum[i];
    S.s.excl[tid] += before;
  }
  if (tid == 0) {
    uint32_t ssum = 0;
    for (uint32_t i = 0; i < SLICE / WAVE; ++i) ssum += S.s.wsum[i];
    S.s.excl[SLICE] = ssum;
    if (sl == NS - 1) {
      uint64_t total = 0;
      for (uint32_t i = 0; i < NT / WAVE; ++i) total += S.s.tot[i];
      ctl->total = total;
      ctl->limit = total < fc.limit ? total : fc.limit;
    }
  }
  __syncthreads();

  // 2. the slice's runs: wave w writes bins [16 w, 16 w + 16) of the slice
  const uint32_t b0 = 16 * wv;
  const uint64_t wstart = spre + S.s.excl[b0];
  const uint64_t wtot = S.s.excl[b0 + 16] - S.s.excl[b0];
  auto count = [&](uint32_t) -> uint32_t { return lane < 16 ? S.s.cnt[b0 + lane] : 0u; };
  wave_fill(S.s.wbuf[wv], out, wstart, wtot, sbase + b0, 1, count, fc);
}

}  // namespace ds
