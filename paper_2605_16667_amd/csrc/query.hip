// libdialsort: queries on a device-resident histogram H, answered without the
// ordered projection.  H is the canonical ordered state (Sec. 3.3, the
// paragraph on the canonical ordered state): frequency(k) and presence(k) read
// one bin; range-count(a, b) and select(r) read the running count
// P[k] = H[0] + ... + H[k-1], built once by a single-pass scan.
//
// Kernels
//   k_query_freq, k_query_presence: one query per thread, a gather from H.
//   k_prefix: tiles of 4096 bins, striped loads transposed through LDS into
//     16 consecutive bins per thread, a block scan, and a decoupled look-back
//     across tiles taken in ticket order (forward progress for any grid), then
//     coalesced uint64 stores of P.  H is read once and P written once.
//   k_query_range: P[min(b, U)] - P[min(a, b, U)].
//   k_query_select: a binary search of r in P (33 dependent loads at most).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/dialsort.h"
#include "common.hpp"
#include "host_common.hpp"
#include "scan_fill.hpp"

using namespace ds;
using namespace dsh;

namespace {

constexpr int Q_NT = 256;
constexpr int PF_NT = 256;
constexpr int PF_VPT = 16;
constexpr uint64_t PF_TB = (uint64_t)PF_NT * PF_VPT;  // bins per scan tile

__global__ __launch_bounds__(Q_NT) void k_query_freq(const uint32_t* __restrict__ H, uint64_t U,
                                                     const uint32_t* __restrict__ q, uint64_t nq,
                                                     uint32_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)Q_NT + threadIdx.x; i < nq; i += (uint64_t)gridDim.x * Q_NT) {
    const uint32_t k = q[i];
    out[i] = (uint64_t)k < U ? H[k] : 0u;
  }
}

__global__ __launch_bounds__(Q_NT) void k_query_presence(const uint32_t* __restrict__ H, uint64_t U,
                                                         const uint32_t* __restrict__ q, uint64_t nq,
                                                         uint8_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)Q_NT + threadIdx.x; i < nq; i += (uint64_t)gridDim.x * Q_NT) {
    const uint32_t k = q[i];
    out[i] = ((uint64_t)k < U && H[k] > 0u) ? 1u : 0u;
  }
}

// Workspace of the prefix scan: a ticket word, then one look-back state per tile.
__global__ void k_prefix_init(uint32_t* ticket, uint64_t* state, uint64_t ntiles) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (tid == 0) *ticket = 0;
  for (uint64_t i = tid; i < ntiles; i += (uint64_t)gridDim.x * blockDim.x) state[i] = 0;
}

// P[k] = H[0] + ... + H[k-1] for k in [0, U], saturating at 2^62 - 1.
__global__ __launch_bounds__(PF_NT) void k_prefix(const uint32_t* __restrict__ H, uint64_t U,
                                                  uint64_t* __restrict__ P, uint32_t* ticket, uint64_t* state) {
  constexpr int TB = PF_NT * PF_VPT;
  constexpr int PADW = TB + TB / 32;
  __shared__ uint32_t tr[PADW];
  __shared__ uint64_t out64[TB + TB / 32];
  __shared__ uint64_t scan_tmp[PF_NT / WAVE + 1];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const uint64_t t = s_tile;
  const uint64_t base = t * (uint64_t)TB;
  // striped loads (coalesced), then thread tid owns bins base + tid*VPT + j;
  // a whole tile loads without bounds tests, so that all its loads are in
  // flight together
  const bool whole = base + TB <= U;
  if (whole) {
    uint32_t h[PF_VPT];
#pragma unroll
    for (int j = 0; j < PF_VPT; ++j) h[j] = H[base + (uint64_t)j * PF_NT + tid];
#pragma unroll
    for (int j = 0; j < PF_VPT; ++j) {
      const uint32_t p = j * PF_NT + tid;
      tr[p + (p >> 5)] = h[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < PF_VPT; ++j) {
      const uint64_t k = base + (uint64_t)j * PF_NT + tid;
      const uint32_t p = j * PF_NT + tid;
      tr[p + (p >> 5)] = k < U ? H[k] : 0u;
    }
  }
  __syncthreads();
  uint32_t v[PF_VPT];
  uint64_t tsum = 0;
#pragma unroll
  for (int j = 0; j < PF_VPT; ++j) {
    const uint32_t p = tid * PF_VPT + j;
    v[j] = tr[p + (p >> 5)];
    tsum += v[j];
  }
  uint64_t agg;
  const uint64_t texcl = block_exclusive_sum<PF_NT>(tsum, scan_tmp, &agg);
  const uint64_t agg_sat = agg > LB_VAL ? LB_VAL : agg;
  if (tid < WAVE) {
    if (t == 0) {
      if (tid == 0) { st_release_u64(&state[0], LB_FLAG_P | agg_sat); s_prefix = 0; }
    } else {
      if (tid == 0) st_release_u64(&state[t], LB_FLAG_A | agg_sat);
      const uint64_t pre = lookback(state, t);
      if (tid == 0) {
        st_release_u64(&state[t], LB_FLAG_P | sat_add(pre, agg_sat));
        s_prefix = pre;
      }
    }
  }
  __syncthreads();
  // running counts of the thread's bins, back to the striped layout
  uint64_t run = sat_add(s_prefix, texcl);
#pragma unroll
  for (int j = 0; j < PF_VPT; ++j) {
    const uint32_t p = tid * PF_VPT + j;
    out64[p + (p >> 5)] = run;
    run = sat_add(run, v[j]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < PF_VPT; ++j) {
    const uint64_t k = base + (uint64_t)j * PF_NT + tid;
    const uint32_t p = j * PF_NT + tid;
    if (whole || k < U) P[k] = out64[p + (p >> 5)];
  }
  // the tile holding bin U - 1 also writes P[U], the total
  if (base <= U - 1 && U - 1 < base + TB && tid == 0) P[U] = sat_add(s_prefix, agg_sat);
}

__global__ __launch_bounds__(Q_NT) void k_query_range(const uint64_t* __restrict__ P, uint64_t U,
                                                      const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                      uint64_t nq, uint64_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)Q_NT + threadIdx.x; i < nq; i += (uint64_t)gridDim.x * Q_NT) {
    const uint64_t hi = b[i] < U ? b[i] : U;
    uint64_t lo = a[i] < U ? a[i] : U;
    lo = lo < hi ? lo : hi;
    out[i] = P[hi] - P[lo];
  }
}

// The element at position r of the ordered projection: the k with
// P[k] <= r < P[k + 1], found by bisection over P[0 .. U].
__global__ __launch_bounds__(Q_NT) void k_query_select(const uint64_t* __restrict__ P, uint64_t U,
                                                       const uint64_t* __restrict__ r, uint64_t nq,
                                                       uint32_t* __restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)Q_NT + threadIdx.x; i < nq; i += (uint64_t)gridDim.x * Q_NT) {
    const uint64_t x = r[i];
    if (x >= P[U]) {
      out[i] = 0xFFFFFFFFu;
      continue;
    }
    // invariant: P[lo] <= x < P[hi]
    uint64_t lo = 0, hi = U;
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (P[mid] <= x) lo = mid; else hi = mid;
    }
    out[i] = (uint32_t)lo;
  }
}

uint32_t query_grid(uint64_t nq) { return (uint32_t)std::min<uint64_t>(cdiv(nq, Q_NT), 256 * 16); }

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

size_t prefix_ws_bytes(uint64_t U) { return ALIGN + align_up(cdiv(U, PF_TB) * 8, ALIGN) + ALIGN; }

}  // namespace

namespace dsh {

// The running count P of H (U + 1 entries) with the workspace laid out by
// prefix_ws_bytes; arguments already checked.
dialsort_status launch_prefix(const uint32_t* H, uint64_t U, uint64_t* P, void* ws, hipStream_t stream) {
  char* base = ws_base(ws);
  uint32_t* ticket = (uint32_t*)base;
  uint64_t* state = (uint64_t*)(base + ALIGN);
  const uint64_t ntiles = cdiv(U, PF_TB);
  DS_LAUNCH(k_prefix_init, dim3((uint32_t)std::min<uint64_t>(cdiv(ntiles + 1, 256), 1024)), dim3(256), stream,
            ticket, state, ntiles);
  DS_LAUNCH(k_prefix, dim3((uint32_t)ntiles), dim3(PF_NT), stream, H, U, P, ticket, state);
  return DIALSORT_OK;
}

}  // namespace dsh

extern "C" {

dialsort_status dialsort_query_frequency(const uint32_t* H, uint64_t U, const uint32_t* q, uint64_t nq,
                                         uint32_t* out, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (nq && (!q || !out))) return DIALSORT_EINVAL;
  if (!aligned4(H) || !aligned4(q) || !aligned4(out)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  if (nq) DS_LAUNCH(k_query_freq, dim3(query_grid(nq)), dim3(Q_NT), stream, H, U, q, nq, out);
  return DIALSORT_OK;
}

dialsort_status dialsort_query_presence(const uint32_t* H, uint64_t U, const uint32_t* q, uint64_t nq,
                                        uint8_t* out, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (nq && (!q || !out))) return DIALSORT_EINVAL;
  if (!aligned4(H) || !aligned4(q)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  if (nq) DS_LAUNCH(k_query_presence, dim3(query_grid(nq)), dim3(Q_NT), stream, H, U, q, nq, out);
  return DIALSORT_OK;
}

size_t dialsort_prefix_workspace_bytes(uint64_t U) { return U == 0 || U > U_MAX ? 0 : prefix_ws_bytes(U); }

dialsort_status dialsort_prefix(const uint32_t* H, uint64_t U, uint64_t* P, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || !P) return DIALSORT_EINVAL;
  if (!aligned4(H) || !aligned8(P)) return DIALSORT_EINVAL;
  if (overlap(H, U * 4, P, (U + 1) * 8)) return DIALSORT_EINVAL;
  if (!ws || ws_bytes < prefix_ws_bytes(U)) return DIALSORT_EWORKSPACE;
  CallScope scope(stream);
  return dsh::launch_prefix(H, U, P, ws, stream);
}

dialsort_status dialsort_query_range_count(const uint64_t* P, uint64_t U, const uint64_t* a, const uint64_t* b,
                                           uint64_t nq, uint64_t* out, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !P || (nq && (!a || !b || !out))) return DIALSORT_EINVAL;
  if (!aligned8(P) || !aligned8(a) || !aligned8(b) || !aligned8(out)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  if (nq) DS_LAUNCH(k_query_range, dim3(query_grid(nq)), dim3(Q_NT), stream, P, U, a, b, nq, out);
  return DIALSORT_OK;
}

dialsort_status dialsort_query_select(const uint64_t* P, uint64_t U, const uint64_t* r, uint64_t nq,
                                      uint32_t* out, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !P || (nq && (!r || !out))) return DIALSORT_EINVAL;
  if (!aligned8(P) || !aligned8(r) || !aligned4(out)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  if (nq) DS_LAUNCH(k_query_select, dim3(query_grid(nq)), dim3(Q_NT), stream, P, U, r, nq, out);
  return DIALSORT_OK;
}

}  // extern "C"
