// Ordered projection (DialSort Sec. 3.3, Eq. (2)) written straight from counts
// a wave already holds: bin k is emitted H[k] times, bins in ascending order.
//
// A wave owns a stretch of consecutive bins and the output positions
// [ws0, we0) of their runs.  It takes the bins 64 at a time, one per lane; a
// wave scan of the counts places every run, each lane writes its run into a
// window of WIN_POS positions in LDS, aligned to 16-byte output quads, and a
// full window goes out with one 16-byte store per lane.  A step holding a run
// longer than WIN_LONG writes its runs one by one with the whole wave, the
// aligned interior of a long run straight to memory.  LDS operations of one
// wave take effect in program order, so the window needs no fence.
#pragma once

#include "common.hpp"

namespace ds {

constexpr uint32_t WIN_POS = 4 * WAVE;  // default window: one 16-byte quad per lane
constexpr uint32_t WIN_LONG = 64;       // longer runs take the wave-wide path

// How runs are written: bin k holds lo + k, or lut[k] when lut is set (the
// table phi^-1 of Sec. 3.4); oal: out is 16-byte aligned; nts: the 16-byte
// stores are non-temporal (outputs far larger than the caches); limit: the
// output's length -- no store reaches past it, whatever the counts say.
struct FillCfg {
  uint32_t lo;
  const uint32_t* lut;
  uint64_t limit;
  bool oal, nts;
};

__device__ __forceinline__ void store_quad(uint32_t* __restrict__ out, uint64_t p, uint4 v, bool nts) {
  if (nts) {
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    const u32x4_t x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4_t*>(out + p));
  } else {
    *reinterpret_cast<uint4*>(out + p) = v;
  }
}

// Write window positions [bb + 4 lane, +4) that lie in [lo, hi) (one quad per
// lane of the first WIN / 4 lanes): a whole quad with one 16-byte store when the
// output is 16-byte aligned, else element by element.
template <uint32_t WIN = WIN_POS>
__device__ __forceinline__ void flush_window(const uint32_t* buf, uint32_t* __restrict__ out, uint64_t bb, uint64_t lo,
                                             uint64_t hi, const FillCfg& fc) {
  static_assert(WIN % 4 == 0 && WIN <= 4 * WAVE, "a window is at most one quad per lane");
  const uint32_t lane = lane_id();
  if (WIN < 4 * WAVE && lane >= WIN / 4) return;
  const uint64_t p = bb + 4ull * lane;
  if (p >= hi || p + 4 <= lo) return;
  const uint4 v = *reinterpret_cast<const uint4*>(buf + 4 * lane);
  if (fc.oal && p >= lo && p + 4 <= hi) {
    store_quad(out, p, v, fc.nts);
  } else {
    if (p >= lo && p < hi) out[p] = v.x;
    if (p + 1 >= lo && p + 1 < hi) out[p + 1] = v.y;
    if (p + 2 >= lo && p + 2 < hi) out[p + 2] = v.z;
    if (p + 3 >= lo && p + 3 < hi) out[p + 3] = v.w;
  }
}

// A wave's output stream: positions [ws0, we0) of out, produced in order
// through the window buf of WIN positions starting at bb (a multiple of 4,
// wave-uniform).
struct WaveOut {
  uint32_t* buf;
  uint64_t bb, ws0, we0;
};

// Run [sk, sk + hk) of value vk (hk > 0; sk >= bb and every position before sk
// is already in the window or written), written by the whole wave: the part
// inside the current window goes to the window; a full window is flushed;
// whole quads of the run past the next window go straight to out.
template <uint32_t WIN = WIN_POS>
__device__ __forceinline__ void wave_run(WaveOut& o, uint32_t* __restrict__ out, uint64_t sk, uint64_t hk,
                                         uint32_t vk, const FillCfg& fc) {
  const uint32_t lane = lane_id();
  const uint64_t end = sk + hk;
  uint64_t p = sk;
  while (p < end) {  // wave-uniform
    const uint64_t wend = o.bb + WIN;
    const uint32_t r0 = (uint32_t)(p - o.bb), r1 = (uint32_t)((end < wend ? end : wend) - o.bb);
    for (uint32_t q = r0 + lane; q < r1; q += WAVE) o.buf[q] = vk;
    if (end < wend) break;
    flush_window<WIN>(o.buf, out, o.bb, o.ws0, wend < o.we0 ? wend : o.we0, fc);
    o.bb = wend;
    p = wend;
    const uint64_t qe = (end < o.we0 ? end : o.we0) & ~3ull;
    if (qe > o.bb + WIN) {
      const uint4 v4 = make_uint4(vk, vk, vk, vk);
      for (uint64_t q = o.bb + 4ull * lane; q < qe; q += 4ull * WAVE) {
        if (fc.oal) {
          store_quad(out, q, v4, fc.nts);
        } else {
          out[q] = vk; out[q + 1] = vk; out[q + 2] = vk; out[q + 3] = vk;
        }
      }
      o.bb = qe;
      p = qe;
    }
  }
}

// The wave writes the runs of `steps` groups of 64 consecutive bins, group j
// holding bins k0 + 64 j + lane; count(j) is this lane's count in group j and
// the group's bins hold wtot keys in all, starting at output position wstart.
// buf: the wave's WIN-word LDS window (16-byte aligned).  Stores stay in
// [wstart, wstart + wtot) cut at fc.limit.
template <uint32_t WIN = WIN_POS, typename CountF>
__device__ __forceinline__ void wave_fill(uint32_t* buf, uint32_t* __restrict__ out, uint64_t wstart, uint64_t wtot,
                                          uint64_t k0, uint32_t steps, CountF count, const FillCfg& fc) {
  if (wtot == 0) return;
  const uint32_t lane = lane_id();
  WaveOut o;
  o.buf = buf;
  o.we0 = wstart + wtot < fc.limit ? wstart + wtot : fc.limit;
  o.ws0 = wstart < o.we0 ? wstart : o.we0;
  o.bb = wstart & ~3ull;
  uint64_t wpos = wstart;  // wave-uniform
#pragma unroll 1
  for (uint32_t j = 0; j < steps; ++j) {
    const uint32_t h = count(j);
    const uint32_t incl = wave_inclusive_sum(h);
    const uint32_t tot = (uint32_t)__shfl((int)incl, WAVE - 1, WAVE);
    if (tot == 0) continue;
    const uint64_t k = k0 + 64ull * j + lane;
    uint32_t v = (uint32_t)k + fc.lo;
    if (fc.lut) v = h ? fc.lut[k] : 0u;
    if (wave_max(h) <= WIN_LONG) {
      // this lane's run: window positions [rs, rs + h) relative to the window
      // base (they fit 32 bits: a step covers at most 64 runs of WIN_LONG);
      // the step ends at rend
      int32_t rs = (int32_t)(wpos - o.bb) + (int32_t)(incl - h);
      int32_t rend = (int32_t)(wpos - o.bb) + (int32_t)tot;
      for (;;) {
        const int32_t a = rs > 0 ? rs : 0;
        const int32_t z = rs + (int32_t)h < (int32_t)WIN ? rs + (int32_t)h : (int32_t)WIN;
        for (int32_t p = a; p < z; ++p) o.buf[p] = v;
        if (rend < (int32_t)WIN) break;
        flush_window<WIN>(o.buf, out, o.bb, o.ws0, o.bb + WIN < o.we0 ? o.bb + WIN : o.we0, fc);
        o.bb += WIN;
        rs -= (int32_t)WIN;
        rend -= (int32_t)WIN;
        if (rend == 0) break;
      }
      wpos += tot;
    } else {
      // a long run in this step: its runs one by one, the whole wave writing
      const uint32_t rel = incl - h;
      uint64_t m = __ballot(h > 0);
      while (m) {
        const uint32_t kk = (uint32_t)__ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const uint32_t hk = (uint32_t)__builtin_amdgcn_readlane((int)h, (int)kk);
        const uint32_t rk = (uint32_t)__builtin_amdgcn_readlane((int)rel, (int)kk);
        const uint32_t vk = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)kk);
        wave_run<WIN>(o, out, wpos + rk, hk, vk, fc);
      }
      wpos += tot;
    }
  }
  // the last, partial window
  flush_window<WIN>(o.buf, out, o.bb, o.ws0, o.we0, fc);
}

}  // namespace ds
