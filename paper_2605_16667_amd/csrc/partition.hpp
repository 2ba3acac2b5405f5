// U-range-partitioned ingestion for universes larger than one workgroup's LDS.
//
// The paper leaves large universes to a "hierarchical" scheme it lists as future
// work (Sec. 16 and Sec. 17); this two-pass design is ours.  The universe is cut
// into B buckets of W = 2^15 consecutive keys (bucket of x = x >> 15).
//
// Pass 1 (k_partition): workgroup t takes tile t of TK = 32768 keys, ranks every
// key inside its bucket with LDS atomics (after the wavefront equality merge),
// and writes the tile's keys grouped by bucket as uint16 bucket-relative keys
// (x & 0x7FFF) into its own slice of the staging buffer, plus the tile's B+1
// segment starts.  Staging stays tile-major, so every write is a coalesced
// 16-byte store and no global counter is needed.
//
// Pass 2 (k_bucket): workgroup b gathers segment b of every tile (16-lane groups
// each read 8-byte words of one segment), counts the relative keys into an LDS
// histogram of W bins, and stores bins [b*W, min((b+1)*W, U)) of H.  H is written
// exactly once with plain stores: no zeroing, no global atomics.  Buckets are
// mapped so that each XCD (blockIdx mod 8) takes a contiguous range of buckets,
// which keeps neighbouring segments and segment-table lines in one L2.
#pragma once

#include "common.hpp"
#include "crn_wave.hpp"
#include "hist_lds.hpp"

namespace ds {

constexpr int PART_LOG2W = 15;
constexpr uint32_t PART_W = 1u << PART_LOG2W;
constexpr int PART_TK = 32768;   // keys per pass-1 tile (segment starts fit in uint16)
constexpr int PART_NT = 1024;
constexpr uint32_t PART_BMAX = 8192;

// seg: T rows of `bstride` uint16 (bstride >= B + 1, multiple of 8).
template <int AGG, bool ALIGNED>
__global__ __launch_bounds__(PART_NT) void k_partition(const uint32_t* __restrict__ keys, uint64_t n, uint32_t umax,
                                                       uint32_t B, uint16_t* __restrict__ staging,
                                                       uint16_t* __restrict__ seg, uint32_t bstride, Ctl* ctl) {
  constexpr int GPT = PART_TK / 4 / PART_NT;  // key groups of 4 per thread
  __shared__ uint32_t cnt[PART_BMAX + 1];
  __shared__ __align__(16) uint16_t stage[PART_TK];
  __shared__ uint32_t scan_tmp[PART_NT / WAVE + 1];
  const uint32_t tid = threadIdx.x;
  const uint64_t tb = (uint64_t)blockIdx.x * PART_TK;
  const uint64_t te = tb + PART_TK < n ? tb + PART_TK : n;

  for (uint32_t i = tid; i <= B; i += PART_NT) cnt[i] = 0;
  __syncthreads();

  uint32_t v[GPT][4];
  uint32_t rk[GPT][4];
  bool okf[GPT][4];
  bool bad = false;
  WaveAgg st;
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    const uint32_t c = load_group<ALIGNED>(keys, tb + ((uint64_t)u * PART_NT + tid) * 4, te, v[u]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool valid = (uint32_t)i < c;
      const bool ok = valid && v[u][i] <= umax;
      bad |= valid && !ok;
      okf[u][i] = ok;
      rk[u][i] = wave_rank<AGG>(cnt, ok ? (v[u][i] >> PART_LOG2W) : 0u, ok, st);
    }
  }
  if (__syncthreads_or(bad) && tid == 0) set_status(ctl, ST_RANGE);

  // exclusive scan of the B+1 counters (counter B stays 0, so cnt[B] becomes the
  // number of valid keys); each thread owns a run of CPT counters
  constexpr int CPT = (PART_BMAX + 1 + PART_NT - 1) / PART_NT;
  uint32_t loc[CPT];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    loc[j] = i <= B ? cnt[i] : 0;
    sum += loc[j];
  }
  uint32_t total;
  uint32_t pre = block_exclusive_sum<PART_NT>(sum, scan_tmp, &total);
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const uint32_t i = tid * CPT + j;
    if (i <= B) cnt[i] = pre;
    pre += loc[j];
  }
  __syncthreads();

  // place the relative keys of valid keys in bucket order
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (okf[u][i]) {
        const uint32_t x = v[u][i];
        stage[cnt[x >> PART_LOG2W] + rk[u][i]] = (uint16_t)(x & (PART_W - 1));
      }
    }
  }
  __syncthreads();

  // tile slice of staging: the valid keys, bucket-major, as 16-byte stores
  const uint32_t nvalid = cnt[B];
  uint16_t* dst = staging + tb;
  const uint32_t n8 = (nvalid + 7) / 8;
  for (uint32_t i = tid; i < n8; i += PART_NT)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(stage)[i];
  uint16_t* srow = seg + (uint64_t)blockIdx.x * bstride;
  for (uint32_t i = tid; i <= B; i += PART_NT) srow[i] = (uint16_t)cnt[i];
}

// Pass 2.  T tiles; H receives bins [b*W, min((b+1)*W, U)).
template <int AGG, bool HALIGNED>
__global__ __launch_bounds__(PART_NT) void k_bucket(const uint16_t* __restrict__ staging,
                                                    const uint16_t* __restrict__ seg, uint32_t bstride,
                                                    uint32_t T, uint32_t B, uint64_t U, uint32_t* __restrict__ H) {
  __shared__ __align__(16) uint32_t s[PART_W];
  const uint32_t tid = threadIdx.x;
  // XCD-aware bucket order: blocks are dispatched round-robin over 8 XCDs
  uint32_t b = blockIdx.x;
  if ((B & 7u) == 0) b = (blockIdx.x & 7u) * (B >> 3) + (blockIdx.x >> 3);

  for (uint32_t i = tid; i < PART_W; i += PART_NT) s[i] = 0;
  __syncthreads();

  Lds32Emit emit{s};
  WaveAgg st;
  constexpr uint32_t NG = PART_NT / 16;  // 16-lane groups
  const uint32_t gid = tid >> 4, l16 = tid & 15;
  uint32_t t = gid;
  uint64_t q = 0, qlo = 0, qhi = 0;  // uint16 indices into staging
  auto open_tile = [&](uint32_t tt) {
    const uint16_t* row = seg + (uint64_t)tt * bstride;
    const uint64_t base = (uint64_t)tt * PART_TK;
    qlo = base + row[b];
    qhi = base + row[b + 1];
    q = (qlo & ~3ull) + 4ull * l16;
  };
  if (t < T) open_tile(t);
  for (;;) {
    while (t < T && q >= qhi) {
      t += NG;
      if (t < T) open_tile(t);
    }
    const bool has = t < T;
    if (!__any(has)) break;
    uint2 w = make_uint2(0, 0);
    if (has) w = *reinterpret_cast<const uint2*>(staging + q);
    const uint32_t r[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool ok = has && (q + i >= qlo) && (q + i < qhi);
      wave_merge<AGG>(r[i], ok, st, emit);
    }
    q += 64;
  }
  __syncthreads();

  const uint64_t hb = (uint64_t)b * PART_W;
  const uint32_t cnt = (uint32_t)(U - hb < PART_W ? U - hb : PART_W);
  if (HALIGNED && cnt == PART_W) {
    for (uint32_t i = tid; i < PART_W / 4; i += PART_NT)
      reinterpret_cast<uint4*>(H + hb)[i] = reinterpret_cast<const uint4*>(s)[i];
  } else {
    for (uint32_t i = tid; i < cnt; i += PART_NT) H[hb + i] = s[i];
  }
}

}  // namespace ds
