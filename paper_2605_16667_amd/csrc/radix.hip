// libdialsort: DialSort-Radix (Sec. 8, "Full int32 range") for the whole
// 32-bit key range: LSD, base 256, four passes, no order comparison.  Each
// pass is the method on one 8-bit digit: the digits are counted (Eq. (1)), the
// running count over the digits and over the tiles before a tile gives where
// that tile's keys of each digit go (the positions of Eq. (2)), and every key
// is placed, in input order within its digit, at that position.  Placement is
// stable, so the passes compose into the sort.  Signed keys go through
// phi(x) = x with the sign bit flipped (Sec. 3.4) on the first load and back on
// the last store.
//
// Kernels
//   k_rdx_init: clears the digit counts, the tile tickets and the tile states.
//   k_rdx_hist: one read of the keys counts all four digits at once into LDS
//     histograms, flushed with one atomic per nonzero bin per block.
//   k_rdx_bases: the running count of each digit histogram (where digit d
//     starts in the output of its pass).
//   k_rdx_pass (one launch per digit): tiles of TK keys taken in ticket order.
//     Each wave ranks its own TK / NW consecutive keys stably per digit (a
//     per-wave match mask and digit counter in LDS); the wave counts
//     give the tile's digit counts, which are published at once; each digit's
//     start for this tile then comes from a decoupled look-back over the
//     previous tiles' published counts (one thread per digit).  Keys are
//     staged in LDS in (digit, input) order and written run by run:
//     consecutive keys of a digit go to consecutive positions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/dialsort.h"
#include "common.hpp"
#include "host_common.hpp"

using namespace ds;
using namespace dsh;

namespace {

constexpr int RX_NT = 1024;              // threads per pass block
constexpr int RX_R = 12;                 // keys per thread
constexpr int RX_TK = RX_NT * RX_R;      // keys per tile
constexpr int RX_HIST_NT = 512;
constexpr int RX_HIST_UNROLL = 8;
constexpr uint32_t RX_HIST_BLOCKS = 512;

__device__ __forceinline__ uint32_t rx_digit(uint32_t x, int shift) { return (x >> shift) & 255u; }

// Tile state of one digit: (tag << 32) | count.  Pass p uses tag 2p + 1 for
// "this tile's count of the digit" and 2p + 2 for "count of the digit over
// tiles 0..t inclusive"; a smaller tag (0 after the clear, or pass p - 1's)
// means not yet published in this pass.
__device__ __forceinline__ uint64_t rx_state(uint32_t tag, uint32_t v) { return ((uint64_t)tag << 32) | v; }

__global__ __launch_bounds__(256) void k_rdx_init(uint64_t* __restrict__ state, uint64_t m, uint32_t* __restrict__ small,
                                                  uint32_t nsmall) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (uint64_t i = g; i < m; i += stride) state[i] = 0;
  for (uint64_t i = g; i < nsmall; i += stride) small[i] = 0;
}

// Block b counts keys [b * per, min(n, (b + 1) * per)) for all four digits.
__global__ __launch_bounds__(RX_HIST_NT) void k_rdx_hist(const uint32_t* __restrict__ src, uint64_t n, uint64_t per,
                                                         uint32_t flip, uint32_t* __restrict__ gh) {
  __shared__ uint32_t h[4 * 256];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < 4 * 256; i += RX_HIST_NT) h[i] = 0;
  __syncthreads();
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = std::min<uint64_t>(n, b0 + per);
  for (uint64_t i = b0 + tid; i < b1; i += (uint64_t)RX_HIST_NT * RX_HIST_UNROLL) {
    // clamped, unconditional loads (b1 > b0: every block has keys)
    uint32_t v[RX_HIST_UNROLL];
#pragma unroll
    for (int k = 0; k < RX_HIST_UNROLL; ++k) v[k] = src[std::min(i + (uint64_t)k * RX_HIST_NT, b1 - 1)] ^ flip;
#pragma unroll
    for (int k = 0; k < RX_HIST_UNROLL; ++k) {
      if (i + (uint64_t)k * RX_HIST_NT < b1) {
        atomicAdd(&h[v[k] & 255u], 1u);
        atomicAdd(&h[256 + ((v[k] >> 8) & 255u)], 1u);
        atomicAdd(&h[512 + ((v[k] >> 16) & 255u)], 1u);
        atomicAdd(&h[768 + (v[k] >> 24)], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < 4 * 256; i += RX_HIST_NT)
    if (h[i]) atomicAdd(&gh[i], h[i]);
}

// Block p: gb[p * 256 + d] = sum of gh[p * 256 + e] over e < d.
__global__ __launch_bounds__(256) void k_rdx_bases(const uint32_t* __restrict__ gh, uint32_t* __restrict__ gb) {
  __shared__ uint32_t tmp[256 / WAVE + 1];
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  uint32_t total;
  gb[i] = block_exclusive_sum<256>(gh[i], tmp, &total);
}

// One pass over digit (x >> shift) & 255.  gbase: where each digit starts in
// dst; state: 256 tile states per tile (tile-major); ticket: tile counter.
template <int NT, int R>
__global__ __launch_bounds__(NT) void k_rdx_pass(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                 uint64_t n, int shift, uint32_t flip_in, uint32_t flip_out,
                                                 const uint32_t* __restrict__ gbase, uint64_t* __restrict__ state,
                                                 uint32_t* __restrict__ ticket, uint32_t tag) {
  constexpr int NW = NT / WAVE;
  constexpr int TK = NT * R;
  constexpr int WK = WAVE * R;  // keys of one wave
  static_assert(NT >= 256, "one thread per digit");
  static_assert(NW * 256 * 2 <= TK, "the match masks fit in the stage area");
  // stage holds the per-wave match masks (256 x 64 bits per wave) while the
  // keys are ranked, then the tile's keys in (digit, input) order
  __shared__ __align__(16) uint32_t stage[TK];
  __shared__ uint32_t wc[NW][256];  // per-wave digit counters, then their prefix over waves
  __shared__ uint32_t tstart[256];  // where digit d starts within the tile
  __shared__ uint32_t obase[256];   // output position of tile index 0 for digit d (mod 2^32)
  __shared__ uint32_t scan_tmp[NW + 1];
  __shared__ uint32_t s_t;
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = __builtin_amdgcn_readfirstlane(tid / WAVE);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint64_t* const mk = reinterpret_cast<uint64_t*>(stage) + w * 256;
  if (tid == 0) s_t = atomicAdd(ticket, 1u);
  for (uint32_t i = tid; i < NW * 256; i += NT) {
    (&wc[0][0])[i] = 0;
    reinterpret_cast<uint64_t*>(stage)[i] = 0;
  }
  __syncthreads();
  const uint32_t t = s_t;
  // wave w owns keys [t * TK + w * WK, + WK): round r, lane l is key r * 64 + l
  const uint64_t wb = (uint64_t)t * TK + (uint64_t)w * WK;
  const uint32_t lim = wb >= n ? 0u : (uint32_t)std::min<uint64_t>(n - wb, WK);  // valid keys of the wave
  // clamped, unconditional loads, all in flight at once (a wave past the end
  // reads key 0 and discards it)
  const uint32_t* __restrict__ ws = lim ? src + wb : src;
  const uint32_t last = lim ? lim - 1 : 0u;
  uint32_t x[R], pos[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = ws[std::min((uint32_t)r * WAVE + lane, last)] ^ flip_in;
  // Stable rank of each key among the wave's keys of its digit.  The lanes
  // holding digit d in this round find each other through mk[d]: each ORs in
  // its lane bit, then all read the mask back (LDS operations of one wave run
  // in order, so the read sees every lane's OR).  The lowest lane of the group
  // advances the digit's counter and clears the mask after all have read both
  // (one instruction each).
  const uint64_t mybit = 1ull << lane;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool valid = (uint32_t)r * WAVE + lane < lim;
    const uint32_t d = rx_digit(x[r], shift);
    uint64_t peers = 0;
    uint32_t old = 0;
    if (valid) {
      __hip_atomic_fetch_or(&mk[d], mybit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      peers = __hip_atomic_load(&mk[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      old = wc[w][d];
    }
    const uint32_t rk = (uint32_t)__popcll(peers & below);
    pos[r] = old + rk;
    asm volatile("" : "+v"(pos[r]));  // materialise the rank now, so the mask and count die here
    if (valid && rk == 0) {
      wc[w][d] = old + (uint32_t)__popcll(peers);
      __hip_atomic_store(&mk[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
  }
  __syncthreads();
  uint32_t cnt = 0;
  if (tid < 256) {
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      const uint32_t c = wc[v][tid];
      wc[v][tid] = cnt;
      cnt += c;
    }
    st_release_u64(&state[(uint64_t)t * 256 + tid], rx_state(t == 0 ? tag + 1 : tag, cnt));
  }
  uint32_t total;
  const uint32_t ex = block_exclusive_sum<NT>(tid < 256 ? cnt : 0u, scan_tmp, &total);
  if (tid < 256) {
    // decoupled look-back for digit tid over tiles t-1, t-2, ..., four at a time
    uint32_t before = 0;
    int64_t j = (int64_t)t - 1;
    while (j >= 0) {
      uint64_t s[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        s[k] = j - k >= 0 ? ld_acquire_u64(&state[(uint64_t)(j - k) * 256 + tid]) : rx_state(tag + 1, 0);
      // take the states in order up to the first inclusive one (done) or the
      // first one not yet published (stall: read it again)
      int k = 0;
      bool done = false, stall = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (done || stall) continue;
        const uint32_t f = (uint32_t)(s[q] >> 32);
        if (f < tag) {
          stall = true;
          continue;
        }
        before += (uint32_t)s[q];
        done = f == tag + 1;
        k = q + 1;
      }
      if (done) break;
      j -= k;
      if (stall) __builtin_amdgcn_s_sleep(1);
    }
    if (t > 0) st_release_u64(&state[(uint64_t)t * 256 + tid], rx_state(tag + 1, before + cnt));
    tstart[tid] = ex;
    obase[tid] = gbase[tid] + before - ex;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if ((uint32_t)r * WAVE + lane < lim) {
      const uint32_t d = rx_digit(x[r], shift);
      stage[tstart[d] + wc[w][d] + pos[r]] = x[r];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < total; i += NT) {
    const uint32_t v = stage[i];
    dst[obase[rx_digit(v, shift)] + i] = v ^ flip_out;
  }
}

struct RadixLayout {
  uint32_t T = 0;
  uint64_t m = 0;  // tile states: 256 T
  size_t off_tmp = 0, off_state = 0, off_small = 0, bytes = 0;
};

// small: gh (4 x 256 digit counts), gb (4 x 256 digit starts), 4 tickets
constexpr uint32_t RX_SMALL = 4 * 256 * 2 + 4;

RadixLayout radix_layout(uint64_t n) {
  RadixLayout L;
  L.T = (uint32_t)std::max<uint64_t>(1, cdiv(n, RX_TK));
  L.m = 256ull * L.T;
  size_t off = 0;
  L.off_tmp = off; off = align_up(off + std::max<uint64_t>(n, 1) * 4, ALIGN);
  L.off_state = off; off = align_up(off + L.m * 8, ALIGN);
  L.off_small = off; off += RX_SMALL * 4;
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
  uint64_t* state = (uint64_t*)(base + L.off_state);
  uint32_t* gh = (uint32_t*)(base + L.off_small);
  uint32_t* gb = gh + 4 * 256;
  uint32_t* tickets = gb + 4 * 256;
  const uint32_t flip = is_signed ? 0x80000000u : 0u;
  const uint32_t init_grid = (uint32_t)std::min<uint64_t>(2048, std::max<uint64_t>(4, cdiv(L.m, 256 * 4)));
  DS_LAUNCH(k_rdx_init, dim3(init_grid), dim3(256), stream, state, L.m, gh, RX_SMALL);
  const uint64_t per = align_up(cdiv(n, RX_HIST_BLOCKS), (uint64_t)RX_HIST_NT * RX_HIST_UNROLL);
  DS_LAUNCH(k_rdx_hist, dim3((uint32_t)cdiv(n, per)), dim3(RX_HIST_NT), stream, keys, n, per, flip, gh);
  DS_LAUNCH(k_rdx_bases, dim3(4), dim3(256), stream, gh, gb);
  // keys -> tmp -> out -> tmp -> out; the first load and the last store flip
  const uint32_t* src = keys;
  for (int pass = 0; pass < 4; ++pass) {
    uint32_t* dst = (pass & 1) ? out : tmp;
    const uint32_t fin = pass == 0 ? flip : 0u, fout = pass == 3 ? flip : 0u;
    DS_LAUNCH((k_rdx_pass<RX_NT, RX_R>), dim3(L.T), dim3(RX_NT), stream, src, dst, n, 8 * pass, fin, fout,
              gb + 256 * pass, state, tickets + pass, (uint32_t)(2 * pass + 1));
    src = dst;
  }
  return DIALSORT_OK;
}

}  // extern "C"
