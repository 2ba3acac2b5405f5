// libdialsort: the key range of an array, for choosing the offset
// order-isomorphism phi(x) = x - lo of the General Self-Indexing Principle
// (Sec. 3.4): lo = min and U = max - min + 1 give the smallest universe that
// holds the keys (the min-max choice of phi).
//
// Kernels
//   k_range_init: the running pair (min, max) := (2^32 - 1, 0).
//   k_range: grid-stride, clamped unconditional loads (eight in flight per
//     thread), a wave reduction, then a workgroup reduction through LDS and one
//     atomicMin/atomicMax per workgroup (few workgroups, so the two words see
//     few atomics).  Signed keys are compared with their sign bit flipped (then
//     unsigned order is signed order).
//   k_range_fini: flips the pair back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/dialsort.h"
#include "common.hpp"
#include "host_common.hpp"

using namespace ds;
using namespace dsh;

namespace {

constexpr int RG_NT = 1024;
constexpr int RG_UNROLL = 8;
constexpr uint32_t RG_BLOCKS = 512;  // two workgroups per CU

__global__ void k_range_init(uint32_t* mm) {
  if (threadIdx.x == 0) {
    mm[0] = 0xFFFFFFFFu;
    mm[1] = 0u;
  }
}

__global__ __launch_bounds__(RG_NT) void k_range(const uint32_t* __restrict__ keys, uint64_t n, uint32_t flip,
                                                 uint32_t* __restrict__ mm) {
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  const uint64_t step = (uint64_t)gridDim.x * RG_NT * RG_UNROLL;
  for (uint64_t i = (uint64_t)blockIdx.x * RG_NT * RG_UNROLL + threadIdx.x; i < n; i += step) {
    uint32_t v[RG_UNROLL];
#pragma unroll
    for (int k = 0; k < RG_UNROLL; ++k) v[k] = keys[std::min(i + (uint64_t)k * RG_NT, n - 1)] ^ flip;
#pragma unroll
    for (int k = 0; k < RG_UNROLL; ++k) {
      // a clamped load repeats key n - 1, which is in range anyway
      lo = std::min(lo, v[k]);
      hi = std::max(hi, v[k]);
    }
  }
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) {
    lo = std::min(lo, (uint32_t)__shfl_xor(lo, d, WAVE));
    hi = std::max(hi, (uint32_t)__shfl_xor(hi, d, WAVE));
  }
  __shared__ uint32_t red[2][RG_NT / WAVE];
  const uint32_t w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[0][w] = lo;
    red[1][w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t v = 1; v < RG_NT / WAVE; ++v) {
      lo = std::min(lo, red[0][v]);
      hi = std::max(hi, red[1][v]);
    }
    atomicMin(&mm[0], lo);
    atomicMax(&mm[1], hi);
  }
}

__global__ void k_range_fini(uint32_t* mm, uint32_t flip) {
  if (threadIdx.x == 0) {
    mm[0] ^= flip;
    mm[1] ^= flip;
  }
}

}  // namespace

extern "C" {

dialsort_status dialsort_key_range(const uint32_t* keys, uint64_t n, int is_signed, uint32_t* minmax,
                                   hipStream_t stream) {
  if (!minmax || (n && !keys)) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(minmax)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, minmax, 8)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  const uint32_t flip = is_signed ? 0x80000000u : 0u;
  DS_LAUNCH(k_range_init, dim3(1), dim3(64), stream, minmax);
  if (n) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(n, (uint64_t)RG_NT * RG_UNROLL), RG_BLOCKS);
    DS_LAUNCH(k_range, dim3(grid), dim3(RG_NT), stream, keys, n, flip, minmax);
  }
  DS_LAUNCH(k_range_fini, dim3(1), dim3(64), stream, minmax, flip);
  return DIALSORT_OK;
}

}  // extern "C"
