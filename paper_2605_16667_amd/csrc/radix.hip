// libdialsort: DialSort-Radix (Sec. 8, "Full int32 range") for the whole
// 32-bit key range: LSD, base 256, four passes, no order comparison.  Each
// pass is the method on one 8-bit digit: the digits are counted into per-tile
// histograms (Eq. (1)), the running count over (digit, tile) gives where each
// tile's keys of each digit go (the positions of Eq. (2)), and every key is
// placed, in input order within its digit, at that position.  Placement is
// stable, so the passes compose into the sort.  Signed keys go through
// phi(x) = x with the sign bit flipped (Sec. 3.4) on the first load and back on
// the last store.
//
// Kernels (per pass)
//   k_rdx_count: tile of RX_TK keys, one LDS histogram of 256 digits, written
//     digit-major (counts[d * T + t]) so that one scan orders (digit, tile).
//   dialsort_prefix over those 256 T counts (the look-back scan of query.hip).
//   k_rdx_scatter: the tile's keys again, ranked stably within each digit in
//     rounds of 256 (match masks from 8 ballots per wave, wave counts combined
//     in wave order through LDS), staged in LDS in (digit, input) order, then
//     written out run by run: consecutive keys of a digit go to consecutive
//     positions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/dialsort.h"
#include "common.hpp"
#include "host_common.hpp"

using namespace ds;
using namespace dsh;

namespace {

constexpr int RX_NT = 256;
constexpr int RX_R = 16;                 // keys per thread (rounds)
constexpr int RX_TK = RX_NT * RX_R;      // keys per tile
constexpr int RX_NW = RX_NT / WAVE;
constexpr uint32_t RX_NONE = 256;        // digit of a slot past the end

// Key i of the tile sits in round i / RX_NT, thread i % RX_NT, so rounds in
// order and threads in order within a round are the input order.
__device__ __forceinline__ uint32_t rx_digit(uint32_t x, int shift) { return (x >> shift) & 255u; }

__global__ __launch_bounds__(RX_NT) void k_rdx_count(const uint32_t* __restrict__ src, uint64_t n, int shift,
                                                     uint32_t flip, uint32_t* __restrict__ counts, uint32_t T) {
  __shared__ uint32_t cnt[256];
  const uint32_t tid = threadIdx.x, t = blockIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const uint64_t tb = (uint64_t)t * RX_TK;
#pragma unroll
  for (int r = 0; r < RX_R; ++r) {
    const uint64_t i = tb + (uint64_t)r * RX_NT + tid;
    if (i < n) atomicAdd(&cnt[rx_digit(src[i] ^ flip, shift)], 1u);
  }
  __syncthreads();
  counts[(uint64_t)tid * T + t] = cnt[tid];
}

__global__ __launch_bounds__(RX_NT) void k_rdx_scatter(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                       uint64_t n, int shift, uint32_t flip_in, uint32_t flip_out,
                                                       const uint64_t* __restrict__ P, uint32_t T) {
  __shared__ uint32_t stage[RX_TK];
  __shared__ uint32_t wcnt[RX_NW][256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t tstart[256 + 1];
  __shared__ uint32_t scan_tmp[RX_NW + 1];
  const uint32_t tid = threadIdx.x, t = blockIdx.x, lane = lane_id(), w = tid / WAVE;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint64_t tb = (uint64_t)t * RX_TK;
  run[tid] = 0;
#pragma unroll
  for (int v = 0; v < RX_NW; ++v) wcnt[v][tid] = 0;
  uint32_t x[RX_R], dg[RX_R], pos[RX_R];
#pragma unroll
  for (int r = 0; r < RX_R; ++r) {
    const uint64_t i = tb + (uint64_t)r * RX_NT + tid;
    x[r] = i < n ? src[i] ^ flip_in : 0u;
    dg[r] = i < n ? rx_digit(x[r], shift) : RX_NONE;
  }
  __syncthreads();
  // stable rank of every key within its digit, round by round
#pragma unroll
  for (int r = 0; r < RX_R; ++r) {
    const uint32_t d = dg[r];
    const bool valid = d != RX_NONE;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot(((d >> b) & 1u) != 0);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank_w = (uint32_t)__popcll(peers & below);
    const bool leader = valid && rank_w == 0;
    if (leader) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = run[d] + rank_w;
      for (uint32_t v = 0; v < w; ++v) off += wcnt[v][d];
      pos[r] = off;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int v = 0; v < RX_NW; ++v) {
      add += wcnt[v][tid];
      wcnt[v][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
  // where each digit's keys start within the tile
  uint32_t total;
  const uint32_t ex = block_exclusive_sum<RX_NT>(run[tid], scan_tmp, &total);
  tstart[tid] = ex;
  if (tid == 0) tstart[256] = total;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RX_R; ++r)
    if (dg[r] != RX_NONE) stage[tstart[dg[r]] + pos[r]] = x[r];
  __syncthreads();
  // write out in tile order: the keys of digit d go to P[d * T + t] onwards
  for (uint32_t i = tid; i < total; i += RX_NT) {
    const uint32_t v = stage[i];
    const uint32_t d = rx_digit(v, shift);
    dst[P[(uint64_t)d * T + t] + (i - tstart[d])] = v ^ flip_out;
  }
}

struct RadixLayout {
  uint32_t T = 0;
  uint64_t m = 0;  // counters: 256 T
  size_t off_tmp = 0, off_counts = 0, off_P = 0, off_pws = 0, bytes = 0;
};

RadixLayout radix_layout(uint64_t n) {
  RadixLayout L;
  L.T = (uint32_t)std::max<uint64_t>(1, cdiv(n, RX_TK));
  L.m = 256ull * L.T;
  size_t off = 0;
  L.off_tmp = off; off = align_up(off + std::max<uint64_t>(n, 1) * 4, ALIGN);
  L.off_counts = off; off = align_up(off + L.m * 4, ALIGN);
  L.off_P = off; off = align_up(off + (L.m + 1) * 8, ALIGN);
  L.off_pws = off; off += dialsort_prefix_workspace_bytes(L.m);
  L.bytes = off + ALIGN;
  return L;
}

}  // namespace

extern "C" {

size_t dialsort_radix_workspace_bytes(uint64_t n) { return n > N_MAX ? 0 : radix_layout(n).bytes; }

dialsort_status dialsort_sort_radix(const uint32_t* keys, uint64_t n, int is_signed, uint32_t* out, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  if (n && (!keys || !out)) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(out)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (out != keys && overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  const RadixLayout L = radix_layout(n);
  if (!ws || ws_bytes < L.bytes) return DIALSORT_EWORKSPACE;
  CallScope scope(stream);
  if (n == 0) return DIALSORT_OK;
  char* base = ws_base(ws);
  uint32_t* tmp = (uint32_t*)(base + L.off_tmp);
  uint32_t* counts = (uint32_t*)(base + L.off_counts);
  uint64_t* P = (uint64_t*)(base + L.off_P);
  void* pws = base + L.off_pws;
  const uint32_t flip = is_signed ? 0x80000000u : 0u;
  // keys -> tmp -> out -> tmp -> out; the first load and the last store flip
  const uint32_t* src = keys;
  for (int pass = 0; pass < 4; ++pass) {
    uint32_t* dst = (pass & 1) ? out : tmp;
    const uint32_t fin = pass == 0 ? flip : 0u, fout = pass == 3 ? flip : 0u;
    DS_LAUNCH(k_rdx_count, dim3(L.T), dim3(RX_NT), stream, src, n, 8 * pass, fin, counts, L.T);
    DS_TRY(launch_prefix(counts, L.m, P, pws, stream));
    DS_LAUNCH(k_rdx_scatter, dim3(L.T), dim3(RX_NT), stream, src, dst, n, 8 * pass, fin, fout, P, L.T);
    src = dst;
  }
  return DIALSORT_OK;
}

}  // extern "C"
