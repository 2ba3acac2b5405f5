// Batched DialSort: many independent arrays, each with its own n, U, H and
// output, sorted by ONE persistent launch.
//
// Every array is cut into work units of three phases:
//   A  ingestion   -- LDS path (U <= W): chunks of `per` keys, each counted into a
//                     private LDS histogram and written as one partial row (or as
//                     H itself when the array has a single chunk);
//                     partitioned path (U > W): groups of BT_TK-key tiles
//                     (partition_tile, bucket = x >> LOG2W);
//   B  counting    -- LDS path: one unit sums the rows into H and scans it;
//                     partitioned path: groups of buckets (bucket_body), each
//                     writing its H slice and scanning it;
//                     both append the array's fill items (Eq. (2) pieces);
//   C  projection  -- fill units, each taking every F-th item slot of its array.
// The host lists the units phase by phase (all A units of the batch, then all B
// units, then all C units; inside a phase, larger arrays first).  Workgroups take
// units in that order from one ticket counter.  The fill units of the size
// classes that end late in the batch (most of its output) are listed apart and
// run in a second kernel, k_batch_fill, right after this one: fill work needs
// little LDS, and there it runs at many more waves per CU than the fused
// kernel, whose workgroup is sized for the counting units' histograms.  A unit that depends on others
// (B on its array's A units, C on its array's B units) spins on its array's
// completion counter until they are done.  The units it waits for hold smaller
// tickets, so they were taken by workgroups that are already running, and the
// unit with the smallest unfinished ticket never waits: the launch always
// drains, whatever the grid size and however many workgroups are resident.
//
// Publication across workgroups (which may sit on different XCDs, each with its
// own L2): a finished unit fences its stores at agent scope in every thread
// before a barrier, then thread 0 adds to the counter with release semantics; a
// waiting unit acquires the counter in thread 0, and every thread fences at
// agent scope after the barrier before it reads what the counter announced.
#pragma once

#include "common.hpp"
#include "hist_lds.hpp"
#include "partition.hpp"
#include "scan_fill.hpp"

namespace ds {

constexpr uint32_t BT_BMAX = 1024;  // buckets per array on the fused path
constexpr int BT_CL2 = 11;          // fill item span: 2048 positions (one wave)
constexpr int BT_TK = 16384;        // keys per partition tile

enum BatchKind : uint32_t { BA_EMPTY = 0, BA_LDS = 1, BA_PART = 2 };
enum UnitType : uint32_t { UT_HIST = 0, UT_PART = 1, UT_ROWS = 2, UT_BUCKET = 3, UT_FILL = 4 };

// One array of the batch, as planned by the host.
struct BArray {
  const uint32_t* keys;
  uint32_t* H;
  uint32_t* out;
  uint32_t* rows;       // LDS path: partial rows (na x row_stride), or H when na == 1
  uint16_t* staging;    // partitioned path
  uint16_t* seg;
  FillItem* items;
  uint64_t n, U;
  uint64_t per;         // LDS path: keys per chunk (multiple of 4)
  uint64_t row_stride;
  uint32_t kind;
  uint32_t na;          // A pieces: chunks or tiles
  uint32_t nb;          // B pieces: 1 or buckets
  uint32_t nf;          // C units
  uint32_t B, bstride;
  uint32_t item_cap;
  uint32_t pad;
};

// Per-array progress, zeroed before every launch.
struct BState {
  uint32_t a_done;   // A pieces finished
  uint32_t b_done;   // B pieces finished
  uint32_t nitems;   // fill items appended
  uint32_t c_done;   // C units finished
  uint64_t t_done;   // wall clock when the array's last unit finished
  uint32_t status;   // the array's own status bits (ST_*)
  uint32_t pad;
};
static_assert(sizeof(BState) == 32, "state is 32 bytes");

struct BUnit {
  uint32_t array;
  uint32_t type;
  uint32_t first;   // first piece, or first item slot (UT_FILL)
  uint32_t count;   // pieces, or the slot stride (UT_FILL)
};

// Launch-wide control, in the first 256 bytes of the batch workspace (Ctl).
// Ctl::tile_ticket is the unit ticket; Ctl::total receives the launch's start
// time (wall clock) and Ctl::limit the time its last unit finished;
// Ctl::prof[2 t] / [2 t + 1] sum, over the units of type t, the clock ticks
// their workgroups spent working / waiting for other units; Ctl::prof[10]
// sums the busy ticks of the fill units run by k_batch_fill.

template <int NT, int LOG2W>
union BatchSmem {
  BinSmem<NT, LOG2W> bin;
  PartSmem<NT, BT_BMAX, BT_TK> part;
  WaveFillSmem<BT_CL2> fill[NT / WAVE];
};

// Wait until *counter >= need.  Thread 0 polls with relaxed agent-scope loads
// (they read the coherent value without invalidating any cache), then one
// acquire fence makes everything published before the counter's increments
// visible to the whole workgroup (it invalidates this CU's L1 and this XCD's
// L2, which every wave of the workgroup reads through).  Returns the clock
// ticks spent waiting (thread 0).
__device__ __forceinline__ uint64_t unit_wait(const uint32_t* counter, uint32_t need) {
  uint64_t waited = 0;
  if (threadIdx.x == 0) {
    if (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need)
        __builtin_amdgcn_s_sleep(8);
      waited = wall_clock64() - t0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return waited;
}

// Publish the unit's stores and add `add` to counter: every wave waits until
// its own stores are acknowledged, then (after the barrier) thread 0 adds with
// release semantics at agent scope, which writes this XCD's L2 back first.
// Returns the counter's old value in thread 0 (0 elsewhere).
__device__ __forceinline__ uint32_t unit_signal(uint32_t* counter, uint32_t add) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  uint32_t old = 0;
  if (threadIdx.x == 0) old = __hip_atomic_fetch_add(counter, add, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  return old;
}

// The array is complete when its last unit finishes: stamp the time and fold
// its status into the batch's.
__device__ __forceinline__ void mark_done(BState* st, Ctl* ctl) {
  const uint64_t now = wall_clock64();
  st->t_done = now;
  __hip_atomic_fetch_max(&ctl->limit, now, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // every other unit of the array has signalled: see their status bits
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const uint32_t bits = __hip_atomic_load(&st->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (bits) atomicOr(&ctl->status, bits);
}

// Unit bodies.
template <int NT, int LOG2W>
__device__ __forceinline__ void unit_hist(BatchSmem<NT, LOG2W>& S, const BArray* __restrict__ Ap, BState* st,
                                       uint32_t first, uint32_t count, uint32_t* status) {
  const BArray& A = *Ap;
  const uint32_t umax = (uint32_t)(A.U - 1);
  for (uint32_t c = first; c < first + count; ++c) {
    const uint64_t beg = (uint64_t)c * A.per;
    const uint64_t end = beg + A.per < A.n ? beg + A.per : A.n;
    uint32_t* row = A.rows + (uint64_t)c * A.row_stride;
    bool packed = false;
    if constexpr (LOG2W == 16) packed = A.U > 32768u;  // two 16-bit counters per word
    if (packed) {
      if constexpr (LOG2W == 16)
        hist_slab<NT, true, 6, true, 4>(S.bin, A.keys, beg, end, umax, (uint32_t)A.U, row, status);
    } else {
      hist_slab<NT, false, 6, true, 4>(S.bin, A.keys, beg, end, umax, (uint32_t)A.U, row, status);
    }
    __syncthreads();
  }
  unit_signal(&st->a_done, count);
}

template <int NT, int LOG2W>
__device__ __forceinline__ void unit_part(BatchSmem<NT, LOG2W>& S, const BArray* __restrict__ Ap, BState* st,
                                       uint32_t first, uint32_t count, uint32_t* status) {
  const BArray& A = *Ap;
  const uint32_t umax = (uint32_t)(A.U - 1);
  for (uint32_t c = first; c < first + count; ++c)
    partition_tile<NT, BT_BMAX, 3, true, LOG2W, BT_TK>(S.part, A.keys, A.n, umax, A.B, A.staging, A.seg, A.bstride, status,
                                                       c, nullptr);
  unit_signal(&st->a_done, count);
}

template <int NT, int LOG2W>
__device__ __forceinline__ uint64_t unit_rows(BatchSmem<NT, LOG2W>& S, const BArray* __restrict__ Ap, BState* st,
                                       uint32_t* status, Ctl* ctl) {
  const BArray& A = *Ap;
  const uint64_t waited = unit_wait(&st->a_done, A.na);
  // several chunks: sum their rows into H; one chunk wrote H itself; no keys: H := 0
  uint32_t* H_out = A.na != 1 ? A.H : nullptr;
  rows_body<NT, LOG2W, true>(S.bin, A.rows, A.na, A.row_stride, H_out, (uint32_t)A.U, status, &st->nitems, A.items,
                             A.item_cap, BT_CL2);
  const uint32_t old = unit_signal(&st->b_done, 1);
  if (threadIdx.x == 0 && A.nf == 0 && old + 1 == A.nb) mark_done(st, ctl);
  return waited;
}

template <int NT, int LOG2W>
__device__ __forceinline__ uint64_t unit_bucket(BatchSmem<NT, LOG2W>& S, const BArray* __restrict__ Ap, BState* st,
                                         uint32_t first, uint32_t count, uint32_t* status, Ctl* ctl) {
  const BArray& A = *Ap;
  const uint64_t waited = unit_wait(&st->a_done, A.na);
  for (uint32_t b = first; b < first + count; ++b) {
    uint64_t base, total;
    bucket_extent<NT>(S.bin, A.seg, A.bstride, A.na, b, &base, &total);
    BucketPart bp;
    bp.b = b;
    bp.t0 = 0;
    bp.t1 = A.na;
    bp.P = 1;
    bp.base = base;
    bp.acc = nullptr;
    bp.done = nullptr;
    bucket_body<NT, LOG2W, 3, true, true, BT_TK>(S.bin, A.staging, A.seg, A.bstride, A.U, A.H, status, &st->nitems,
                                                 A.items, A.item_cap, BT_CL2, bp);
    __syncthreads();
  }
  const uint32_t old = unit_signal(&st->b_done, count);
  if (threadIdx.x == 0 && A.nf == 0 && old + count == A.nb) mark_done(st, ctl);
  return waited;
}

// The fill items of one fill unit: wave w of the NT / WAVE takes the item
// slots first + stride * (w + NW m).  fill: one LDS window per wave.
template <int NT>
__device__ __forceinline__ void fill_unit_items(WaveFillSmem<BT_CL2>* fill, const BArray& A, const BState* st,
                                                uint32_t first, uint32_t stride, uint32_t* status, Ctl* ctl) {
  const uint32_t ni = st->nitems < A.item_cap ? st->nitems : A.item_cap;
  // a failed invariant (ST_INTERNAL) may leave items unwritten: fill nothing
  const bool failed = (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_INTERNAL) != 0;
  if (failed) return;
  constexpr uint32_t NW = NT / WAVE;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
  const uint64_t step = (uint64_t)stride * NW;
  uint64_t j = first + (uint64_t)stride * w;
  // the wave's next item is loaded while the current one is filled
  FillItem next{};
  if (j < ni) next = A.items[j];
  for (; j < ni; j += step) {
    const FillItem I = next;
    if (j + step < ni) next = A.items[j + step];
    // an item always lies inside its array; anything else is a broken
    // invariant, reported (to the array and to the launch) instead of written
    const bool valid = I.k <= I.klast && I.klast < A.U && I.klast - I.k < FILL_SPAN_MAX && I.o <= I.p0 &&
                       I.p0 < I.p1 && I.p1 <= A.n && I.p1 - (I.p0 & ~3ull) <= (1ull << BT_CL2);
    if (!valid) {
      if (lane_id() == 0) {
        atomicOr(status, ST_INT_ITEM);
        atomicOr(&ctl->status, ST_INT_ITEM);
      }
      continue;
    }
    wave_fill_item<BT_CL2, true, false, true>(fill[w], A.H, A.out, I);
  }
}

template <int NT, int LOG2W>
__device__ __forceinline__ uint64_t unit_fill(BatchSmem<NT, LOG2W>& S, const BArray* __restrict__ Ap, BState* st,
                                       uint32_t first, uint32_t stride, uint32_t* status, Ctl* ctl) {
  const BArray& A = *Ap;
  const uint64_t waited = unit_wait(&st->b_done, A.nb);
  fill_unit_items<NT>(S.fill, A, st, first, stride, status, ctl);
  const uint32_t old = unit_signal(&st->c_done, 1);
  if (threadIdx.x == 0 && old + 1 == A.nf) mark_done(st, ctl);
  return waited;
}

template <int NT, int LOG2W>
__global__ __launch_bounds__(NT) void k_batch(const BArray* __restrict__ arrays, BState* __restrict__ states,
                                              const BUnit* __restrict__ units, uint32_t nunits, Ctl* ctl) {
  __shared__ BatchSmem<NT, LOG2W> S;
  __shared__ uint32_t s_ticket;
  const uint32_t tid = threadIdx.x;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const uint32_t t = atomicAdd(&ctl->tile_ticket, 1u);
      if (t == 0) ctl->total = wall_clock64();
      s_ticket = t;
    }
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= nunits) break;
    const BUnit u = units[t];
    const BArray* A = arrays + u.array;
    BState* st = states + u.array;
    uint32_t* status = &st->status;
    const uint64_t t0 = wall_clock64();
    uint64_t waited = 0;
    switch (u.type) {
      case UT_HIST: unit_hist<NT, LOG2W>(S, A, st, u.first, u.count, status); break;
      case UT_PART: unit_part<NT, LOG2W>(S, A, st, u.first, u.count, status); break;
      case UT_ROWS: waited = unit_rows<NT, LOG2W>(S, A, st, status, ctl); break;
      case UT_BUCKET: waited = unit_bucket<NT, LOG2W>(S, A, st, u.first, u.count, status, ctl); break;
      case UT_FILL: waited = unit_fill<NT, LOG2W>(S, A, st, u.first, u.count, status, ctl); break;
      default:
        if (tid == 0) atomicOr(&ctl->status, ST_INT_UNIT);
        break;
    }
    if (tid == 0 && u.type <= UT_FILL) {
      const uint64_t busy = wall_clock64() - t0 - waited;
      __hip_atomic_fetch_add(&ctl->prof[2 * u.type], busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&ctl->prof[2 * u.type + 1], waited, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The fill units listed after the fused kernel's own: launched on the same
// stream right after k_batch, so every array's counting units have finished
// and their H, items and item counts are visible (kernel boundary); nothing
// here waits.  Small workgroups (NTF threads, one LDS window per wave) keep
// many waves per CU in flight, as the single-array fill does.  A unit's
// completion is counted without release semantics: nothing in the launch reads
// the output, the count only stamps the array's completion time (after the
// unit's stores are acknowledged) and folds its status, whose fill bits also
// go straight to the launch status.
template <int NTF>
__global__ __launch_bounds__(NTF, 8) void k_batch_fill(const BArray* __restrict__ arrays, BState* __restrict__ states,
                                                    const BUnit* __restrict__ units, uint32_t nunits, Ctl* ctl) {
  __shared__ WaveFillSmem<BT_CL2> S[NTF / WAVE];
  __shared__ uint32_t s_ticket;
  const uint32_t tid = threadIdx.x;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_ticket = atomicAdd(&ctl->fill_ticket, 1u);
    __syncthreads();
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= nunits) break;
    const BUnit u = units[t];
    const uint64_t t0 = wall_clock64();
    if (u.type != UT_FILL) {
      if (tid == 0) atomicOr(&ctl->status, ST_INT_UNIT);
      continue;
    }
    const BArray& A = arrays[u.array];
    BState* st = states + u.array;
    fill_unit_items<NTF>(S, A, st, u.first, u.count, &st->status, ctl);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      const uint32_t old = __hip_atomic_fetch_add(&st->c_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1 == A.nf) mark_done(st, ctl);
      __hip_atomic_fetch_add(&ctl->prof[2 * UT_FILL + 2], wall_clock64() - t0, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Clears the launch control block and the per-array states.
static __global__ void k_batch_init(Ctl* ctl, BState* states, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < sizeof(Ctl) / 4) reinterpret_cast<uint32_t*>(ctl)[i] = 0;
  const uint32_t nw = count * (uint32_t)(sizeof(BState) / 4);
  for (uint32_t j = i; j < nw; j += gridDim.x * blockDim.x) reinterpret_cast<uint32_t*>(states)[j] = 0;
}

}  // namespace ds
