// Device helpers shared by the DialSort gfx950 kernels: wavefront primitives,
// block scans, key-slab iteration and the workspace control block.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ds {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Workspace control block (first 256 bytes of every workspace).
// ---------------------------------------------------------------------------
struct Ctl {
  uint32_t status;       // bit 0: a key >= U was seen; bit 1: sum(H) > out_cap
  uint32_t tile_ticket;  // dynamic tile order for the look-back scan
  uint32_t bucket_ticket;
  uint32_t fill_ticket;
  uint64_t total;        // sum(H), saturated at SAT_MAX
  uint64_t limit;        // number of output positions that are written
  uint32_t nitems;       // fill items appended by the scan
  uint32_t pad0;
  uint64_t prof[16];     // batched launch: per unit type, workgroup clock ticks busy / waiting
  uint64_t runs;         // long runs of the scan: (count << 40) | their chunks
  uint32_t pad[20];
};
static_assert(sizeof(Ctl) == 256, "control block is 256 bytes");

constexpr uint32_t ST_RANGE = 1u;
constexpr uint32_t ST_OVERFLOW = 2u;
constexpr uint32_t ST_INTERNAL = 0x80000000u;  // a library invariant failed; with it, one cause bit:
constexpr uint32_t ST_INT_ITEMS = ST_INTERNAL | 0x40000000u;  // fill-item list full
constexpr uint32_t ST_INT_ITEM = ST_INTERNAL | 0x20000000u;   // a fill item outside its array
constexpr uint32_t ST_INT_EVLOG = ST_INTERNAL | 0x10000000u;  // packed-counter event log full
constexpr uint32_t ST_INT_UNIT = ST_INTERNAL | 0x08000000u;   // unknown work unit
constexpr uint32_t ST_INT_WAIT = ST_INTERNAL | 0x04000000u;   // a one-launch sort gave up waiting for its rows
constexpr uint64_t SAT_MAX = (uint64_t(1) << 62) - 1;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t sat_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;  // a, b <= SAT_MAX, so no wrap
  return s > SAT_MAX ? SAT_MAX : s;
}

// ---------------------------------------------------------------------------
// Wavefront scans (64 lanes).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T y = __shfl_up(x, d, WAVE);
    if (lane >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
  return x;
}

// Sum over each 32-lane half of the wave, left in lanes 31 and 63: prefix sums
// within each row of 16 lanes (DPP row shifts, lanes shifted in read 0), then
// row 0's total added into row 1 and row 2's into row 3 (DPP row broadcast of
// lane 15).  Every lane must be active.
__device__ __forceinline__ uint32_t half_wave_sum(uint32_t x) {
  int v = (int)x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1 and 3
  return (uint32_t)v;
}

// Maximum over the wave, in a scalar register (the same in every lane).
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int d = WAVE / 2; d >= 1; d >>= 1) {
    const uint32_t y = __shfl_xor(x, d, WAVE);
    x = y > x ? y : x;
  }
  return __builtin_amdgcn_readfirstlane(x);
}

// Exclusive prefix sum over a block of NT threads.  smem needs NT/64 + 1
// elements.  Returns the exclusive prefix; *total receives the block total.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* smem, T* total) {
  constexpr int NW = NT / WAVE;
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  T inc = wave_inclusive_sum(v);
  if (lane == WAVE - 1) smem[w] = inc;
  __syncthreads();
  if (w == 0) {
    T x = lane < NW ? smem[lane] : T(0);
    T xi = wave_inclusive_sum(x);
    if (lane < NW) smem[lane] = xi - x;
    if (lane == NW - 1) smem[NW] = xi;
  }
  __syncthreads();
  T r = smem[w] + inc - v;
  *total = smem[NW];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Key slabs: the key array is split into an unaligned scalar head (0..3 keys,
// so that the body starts on a 16-byte boundary), a body of uint4 groups and a
// scalar tail.  Work item g of G owns body groups [g*per4, min((g+1)*per4, n4)),
// item 0 also owns the head and item G-1 the tail.
// ---------------------------------------------------------------------------
struct Slabs {
  const uint32_t* keys;
  uint64_t n;
  uint32_t head;       // scalar keys before the aligned body
  uint32_t tail;       // scalar keys after the body
  uint64_t n4;         // uint4 groups in the body
  uint64_t per4;       // groups per work item
};

// Atomically record a status bit in the control block.
__device__ __forceinline__ void set_status(Ctl* ctl, uint32_t bit) { atomicOr(&ctl->status, bit); }

// Agent-scope 64-bit atomic load / store for look-back flags.
__device__ __forceinline__ uint64_t ld_acquire_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace ds
