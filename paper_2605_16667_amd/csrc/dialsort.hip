// libdialsort: host side of the DialSort gfx950 hot path -- argument checks,
// plan selection, workspace layout and kernel launches behind the C ABI of
// include/dialsort.h.
//
// Launch sequences (each starts with k_init, which clears the control block and
// the look-back tile flags, and zeroes H only where H is accumulated with
// atomics -- except an LDS ingestion into partial rows, which clears them
// itself):
//   LDS32 / LDS16 (U <= 65536):  k_hist_lds -> [k_scan: sum rows into H]
//   small LDS sorts:               k_sort_lds alone (counting and scan in one launch)
//   PART (65536 < U <= 2^29):     k_partition -> k_bucket (H, and fill items)
//   GLOBAL (tiny n, or U > 2^29): k_hist_global
//   sort adds                      [k_scan: look-back scan + fill items] -> k_fill
//   reconstruct                    k_init -> k_scan -> k_fill
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/dialsort.h"
#include "common.hpp"
#include "host_common.hpp"
#include "hist_lds.hpp"
#include "partition.hpp"
#include "scan_fill.hpp"
#include "sort_lds.hpp"

using namespace ds;
using namespace dsh;

namespace dsh {
thread_local int g_last_hip_error = 0;
thread_local LaunchLog g_log{nullptr, 0, nullptr, 0, std::vector<const char*>(64, nullptr)};
}  // namespace dsh

namespace {

constexpr int FILL_NT = 256;
constexpr int FILL_CL2 = 11;  // fill items of at most 2048 positions (one wave each)
constexpr uint64_t FILL_NTS_BYTES = uint64_t(64) << 20;  // outputs from 64 MiB on use non-temporal stores
constexpr int SCAN_NT = 256;
constexpr uint64_t PART_NCU = 256;  // compute units of the target (MI355X)
constexpr uint64_t DIRECT_NMAX = 1ull << 24;     // direct projection from the scan: at most this many keys,
constexpr uint64_t DIRECT_PER_TILE = 1ull << 14;  // and at most this many per scan tile on average
constexpr int FUSED_NT = 1024;  // one-launch sort: threads per block
constexpr uint64_t FUSED_PER_SLICE = 1ull << 14;  // one-launch sort: at most this many keys per slice of bins on average

enum Kind { K_EMPTY, K_LDS32S, K_LDS32, K_LDS16, K_PART, K_GLOBAL, K_NONE };

struct Layout {
  Kind kind = K_NONE;
  uint32_t G = 1;        // LDS paths: workgroups (= partial rows)
  uint64_t per = 0;      // LDS paths: keys per workgroup (multiple of 4)
  uint32_t B = 0, T = 0, bstride = 0;  // PART
  uint32_t X = 0;        // PART: extra workgroups for the parts of heavy buckets
  uint64_t chunk = 0;    // PART: keys per part of a heavy bucket
  bool rows_in_ws = false;
  bool row16 = false;    // partial rows hold 16-bit counts, two bins per word (fewer than 2^16 keys per row)
  uint64_t row_stride = 0;
  bool scan = false;     // full projection
  bool direct = false;   // LDS paths, sort: the scan tiles write the output (no fill items)
  bool fused = false;    // LDS paths, sort: k_sort_lds may do the whole sort in one launch
  uint32_t NS = 0;       // its slices of bins
  size_t off_pre = 0, off_flags = 0;  // its per-slab slice prefixes (G x (NS + 1)) and G publication flags
  int scan_vpt = 16;
  uint64_t scan_tiles = 0;
  uint64_t limit = 0;
  uint64_t item_cap = 0, run_cap = 0;
  size_t off_tile = 0, off_items = 0, off_runs = 0, off_rows = 0, off_stage = 0, off_seg = 0, bytes = 0;
  size_t off_z = 0, nz = 0;  // PART: cleared words: bucket-total counters, tile ticket, done counters, scratch
  size_t off_done = 0, off_scratch = 0;
};

// Choose the number of LDS workgroups: enough to stream the keys at full
// bandwidth, few enough that the partial rows stay small next to the keys.
uint32_t choose_G(uint64_t n, uint64_t U, uint32_t gmax, uint64_t max_per) {
  const double BWR = 6.0e12, BWW = 5.0e12, RWG = 25.0e9;
  uint32_t g_lo = (uint32_t)std::max<uint64_t>(1, cdiv(n, max_per));
  uint32_t best = g_lo;
  double best_t = 1e30;
  for (uint32_t g = 1; g <= gmax; g *= 2) {
    uint32_t gg = std::max(g, g_lo);
    // bytes per bin of a partial row: 2 when a row counts fewer than 2^16 keys
    const double rb = gg > 1 && align_up(cdiv(n, gg), 4) < 65536 ? 2.0 : 4.0;
    const double t = 4.0 * n / std::min(BWR, gg * RWG) + gg * U * rb / BWW + gg * U * rb / BWR +
                     (gg > 1 ? (gg / 8.0) * 1.0e-6 * (U < 16384 ? 1.0 : 0.1) : 0.0);
    if (t < best_t) { best_t = t; best = gg; }
  }
  return std::min(best, std::max(g_lo, gmax));
}

Layout plan(uint64_t n, uint64_t U, int mode) {
  Layout L;
  const bool recon = mode == DIALSORT_MODE_RECONSTRUCT;
  L.scan = mode != DIALSORT_MODE_HISTOGRAM;
  L.limit = n;  // sort: n positions; reconstruct: out_cap
  size_t off = ALIGN;  // control block first
  if (recon) {
    L.kind = K_NONE;
  } else if (n == 0) {
    L.kind = K_EMPTY;
  } else if (U > PART_UMAX || (U > 65536 && n < (uint64_t)PART_TK)) {
    L.kind = K_GLOBAL;
  } else if (U <= 4096) {
    L.kind = K_LDS32S;
    L.G = choose_G(n, U, 512, 1ull << 40);
  } else if (U <= 32768) {
    L.kind = K_LDS32;
    L.G = choose_G(n, U, 256, 1ull << 40);
  } else if (U <= 65536) {
    L.kind = K_LDS16;
    L.G = choose_G(n, U, 256, 1ull << 22);
  } else {
    L.kind = K_PART;
    L.B = (uint32_t)cdiv(U, PART_W);
    L.T = (uint32_t)cdiv(n, PART_TK);
    L.bstride = (uint32_t)align_up(L.B + 1, 8);
    // a bucket of more than two chunks is counted by several workgroups; a
    // chunk is the keys per CU of an even spread (at least 2^18)
    L.chunk = std::max<uint64_t>(1ull << 18, cdiv(n, PART_NCU));
    L.X = n > 2 * L.chunk ? (uint32_t)std::min<uint64_t>(cdiv(n, L.chunk), 2 * PART_NCU) : 0;
  }
  if (L.kind == K_LDS32S || L.kind == K_LDS32 || L.kind == K_LDS16) {
    L.per = align_up(cdiv(n, L.G), 4);
    L.G = (uint32_t)cdiv(n, L.per);
    L.rows_in_ws = L.G > 1;
    L.row16 = L.rows_in_ws && L.per < 65536;
    L.row_stride = align_up(U + 1, 64);
  }
  // scan tiles (also used to sum partial rows in histogram mode); the
  // partitioned path projects bucket by bucket and needs no scan
  L.scan_vpt = (L.rows_in_ws && L.G >= 8) ? 1 : 16;
  L.scan_tiles = L.kind == K_PART ? 0 : cdiv(U, (uint64_t)SCAN_NT * L.scan_vpt);
  // a sort whose scan tiles each hold few output positions writes the output
  // from the scan itself: one launch and the fill items fewer
  L.direct = mode == DIALSORT_MODE_SORT && (L.kind == K_LDS32S || L.kind == K_LDS32 || L.kind == K_LDS16) &&
             n <= DIRECT_NMAX && n <= DIRECT_PER_TILE * L.scan_tiles;
  // one launch for the whole sort (k_sort_lds): 16-bit rows, and a slice of
  // bins holds few output positions on average
  if (mode == DIALSORT_MODE_SORT && L.row16) {
    const uint64_t ns = cdiv(U, (uint64_t)SLICE);
    L.fused = ns <= FUSED_SLICES_MAX && n <= DIRECT_NMAX && n <= FUSED_PER_SLICE * ns;
    L.NS = L.fused ? (uint32_t)ns : 0;
  }
  if (L.scan) {
    L.off_tile = off; off = align_up(off + L.scan_tiles * 8, ALIGN);
  }
  if (L.fused) {
    L.off_pre = off; off = align_up(off + (size_t)L.G * (L.NS + 1) * 4, ALIGN);
    L.off_flags = off; off = align_up(off + (size_t)L.G * 8, ALIGN);
  }
  if (L.scan && !L.direct) {
    // one item per chunk of output positions, plus one per span boundary that
    // splits a chunk: spans are the scan tiles, or on the partitioned path the
    // projection tiles of PT_BINS bins and the buckets (two pieces for a bucket
    // counted in two halves)
    L.item_cap = (L.kind == K_PART ? 2ull * L.B + cdiv(U, PT_BINS) : L.scan_tiles) +
                 cdiv(L.limit, 1ull << FILL_CL2) + 2;
    L.off_items = off; off = align_up(off + L.item_cap * sizeof(FillItem), ALIGN);
    // run records of the scan: every recorded run holds more than RUN_MIN of
    // the chunks of C positions
    L.run_cap = L.kind == K_PART ? 0 : cdiv(L.limit, RUN_MIN << FILL_CL2) + 1;
    L.off_runs = off; off = align_up(off + L.run_cap * sizeof(FillRun), ALIGN);
  }
  if (L.rows_in_ws) {
    L.off_rows = off; off = align_up(off + (size_t)L.G * L.row_stride * 4, ALIGN);
  }
  if (L.kind == K_PART) {
    L.off_stage = off; off = align_up(off + (align_up(n, 8) + 16) * 2, ALIGN);
    L.off_seg = off; off = align_up(off + (size_t)L.T * L.bstride * 2, ALIGN);
    // one cleared region: bucket-total counters, done counters, scratch rows
    L.off_z = off;
    L.off_done = off + align_up((size_t)colsum_rows(L.B) * L.B * 4, 64);
    L.off_scratch = L.off_done + align_up(SPLIT_SLOTS * 4, 64);
    off = L.off_scratch + (L.X > 0 ? (size_t)SPLIT_SLOTS * PART_W * 4 : 0);
    L.nz = (off - L.off_z) / 4;
    off = align_up(off, ALIGN);
  }
  L.bytes = off + ALIGN;  // slack for aligning the caller's pointer
  return L;
}

// LDS ingestion into partial rows: the ingestion launch clears the control
// block and the look-back flags itself (k_hist_lds, init), and the scan reads
// the rows' status words, so no clearing launch runs first.
// (Partial rows are U + 1 words at least: word U of a row is free.)
bool fold_init(const Layout& L) {
  return L.rows_in_ws && (L.kind == K_LDS32S || L.kind == K_LDS32 || L.kind == K_LDS16);
}

// k_init: clear the control block, the look-back flags, the bucket-total
// counters, and optionally H.
__global__ void k_init(Ctl* ctl, uint64_t* tiles, uint64_t ntiles, uint32_t* z, uint64_t nz, uint32_t* H,
                       uint64_t nH) {
  const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t* c = reinterpret_cast<uint32_t*>(ctl);
  if (tid < sizeof(Ctl) / 4) c[tid] = 0;
  for (uint64_t i = tid; i < ntiles; i += stride) tiles[i] = 0;
  for (uint64_t i = tid; i < nz; i += stride) z[i] = 0;
  for (uint64_t i = tid; i < nH; i += stride) H[i] = 0;
}

dialsort_status launch_init(char* base, const Layout& L, uint32_t* H, uint64_t nH, hipStream_t s) {
  const uint64_t nz = L.kind == K_PART ? L.nz : 0;
  const uint64_t work = std::max<uint64_t>(std::max<uint64_t>(std::max<uint64_t>(64, L.scan ? L.scan_tiles : 0), nH), nz);
  const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(work, 256), 2048);
  DS_LAUNCH(k_init, dim3(grid), dim3(256), s, (Ctl*)base, (uint64_t*)(base + L.off_tile),
            L.scan ? L.scan_tiles : 0, (uint32_t*)(base + L.off_z), nz, H, nH);
  return DIALSORT_OK;
}

// Ingestion: H (or partial rows) from keys.
dialsort_status launch_ingest(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t lo, uint32_t* H, char* base,
                              const Layout& L, hipStream_t s) {
  Ctl* ctl = (Ctl*)base;
  const uint32_t umax = (uint32_t)(U - 1);
  const bool ka = aligned16(keys);
  uint32_t* rows = L.rows_in_ws ? (uint32_t*)(base + L.off_rows) : H;
  // the LDS ingestion into partial rows also clears what the scan needs
  const uint32_t fi = fold_init(L) ? 1u : 0u;
  uint64_t* clr = (uint64_t*)(base + L.off_tile);
  const uint64_t nclr = fi && L.scan ? L.scan_tiles : 0;
  switch (L.kind) {
    case K_LDS32S:
      if (ka) DS_LAUNCH((k_hist_lds<1024, 4096, false, 8, true, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      else DS_LAUNCH((k_hist_lds<1024, 4096, false, 8, false, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      break;
    case K_LDS32:
      if (ka) DS_LAUNCH((k_hist_lds<1024, 32768, false, 8, true, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      else DS_LAUNCH((k_hist_lds<1024, 32768, false, 8, false, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      break;
    case K_LDS16:
      if (ka) DS_LAUNCH((k_hist_lds<1024, 32768, true, 8, true, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      else DS_LAUNCH((k_hist_lds<1024, 32768, true, 8, false, 4>), dim3(L.G), dim3(1024), s, keys, n, L.per, umax, (uint32_t)U, rows, L.row_stride, ctl, lo, fi, clr, nclr, L.row16 ? 1u : 0u);
      break;
    case K_PART: {
      uint16_t* stg = (uint16_t*)(base + L.off_stage);
      uint16_t* seg = (uint16_t*)(base + L.off_seg);
      SplitPlan plan;
      plan.colsum = (uint32_t*)(base + L.off_z);
      plan.rows = colsum_rows(L.B);
      plan.done = (uint32_t*)(base + L.off_done);
      plan.scratch = (uint32_t*)(base + L.off_scratch);
      plan.chunk = L.chunk;
      plan.X = L.X;
      if (L.B <= 1024) {
        if (ka) DS_LAUNCH((k_partition<1024, 3, true>), dim3(L.T), dim3(P1_NT), s, keys, n, umax, L.B, stg, seg, L.bstride, ctl, plan, lo);
        else DS_LAUNCH((k_partition<1024, 3, false>), dim3(L.T), dim3(P1_NT), s, keys, n, umax, L.B, stg, seg, L.bstride, ctl, plan, lo);
      } else {
        if (ka) DS_LAUNCH((k_partition<PART_BMAX, 3, true>), dim3(L.T), dim3(P1_NT), s, keys, n, umax, L.B, stg, seg, L.bstride, ctl, plan, lo);
        else DS_LAUNCH((k_partition<PART_BMAX, 3, false>), dim3(L.T), dim3(P1_NT), s, keys, n, umax, L.B, stg, seg, L.bstride, ctl, plan, lo);
      }
      FillItem* items = (FillItem*)(base + L.off_items);
      const uint32_t icap = (uint32_t)std::min<uint64_t>(L.item_cap, 0xFFFFFFF0ull);
      const bool ha = aligned16(H);
#define DS_BUCKET(HA, FULL)                                                                                   \
  DS_LAUNCH((k_bucket<3, HA, FULL>), dim3(L.B + L.X), dim3(PART_NT), s, stg, seg, L.bstride, L.T, L.B, U, H, ctl, \
            items, icap, FILL_CL2, plan)
      if (!L.scan) {
        if (ha) DS_BUCKET(true, false); else DS_BUCKET(false, false);
      } else {
        if (ha) DS_BUCKET(true, true); else DS_BUCKET(false, true);
      }
#undef DS_BUCKET
      break;
    }
    case K_GLOBAL: {
      const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(n, 256 * 4), 4096);
      if (ka) DS_LAUNCH((k_hist_global<256, 3, true>), dim3(grid), dim3(256), s, keys, n, umax, H, ctl, lo);
      else DS_LAUNCH((k_hist_global<256, 3, false>), dim3(grid), dim3(256), s, keys, n, umax, H, ctl, lo);
      break;
    }
    default:
      break;
  }
  return DIALSORT_OK;
}

// k_scan over `rows` (nrows rows), writing H when H_out is set.  With
// L.direct (and full) the scan tiles write the sorted output themselves.
dialsort_status launch_scan(const uint32_t* rows, uint32_t nrows, uint64_t row_stride, uint32_t* H_out,
                            uint64_t U, char* base, const Layout& L, bool full, int report_overflow,
                            hipStream_t s, uint32_t* out = nullptr, FillCfg fc = FillCfg{}) {
  Ctl* ctl = (Ctl*)base;
  uint64_t* tiles = (uint64_t*)(base + L.off_tile);
  FillItem* items = (FillItem*)(base + L.off_items);
  const uint32_t icap = (uint32_t)std::min<uint64_t>(L.item_cap, 0xFFFFFFF0ull);
  FillRun* runs = (FillRun*)(base + L.off_runs);
  const uint32_t rcap = (uint32_t)std::min<uint64_t>(L.run_cap, 0xFFFFFFF0ull);
  const dim3 grid((uint32_t)L.scan_tiles);
  // rows are the ingestion's partial rows carrying status words (and, with
  // row16, counts of 16 bits)
  const uint32_t rstat = fold_init(L) && nrows == L.G && row_stride == L.row_stride ? 1u : 0u;
  const uint32_t r16 = rstat && L.row16 ? 1u : 0u;
#define DS_SCAN(VPT, FULL, DIRECT)                                                                                  \
  DS_LAUNCH((k_scan<SCAN_NT, VPT, FULL, DIRECT>), grid, dim3(SCAN_NT), s, rows, nrows, row_stride, H_out, U, ctl, \
            tiles, items, icap, L.limit, FILL_CL2, report_overflow, runs, rcap, out, fc, rstat, r16)
  if (full && L.direct) {
    if (L.scan_vpt == 1) DS_SCAN(1, true, true); else DS_SCAN(16, true, true);
  } else if (full) {
    if (L.scan_vpt == 1) DS_SCAN(1, true, false); else DS_SCAN(16, true, false);
  } else {
    if (L.scan_vpt == 1) DS_SCAN(1, false, false); else DS_SCAN(16, false, false);
  }
#undef DS_SCAN
  return DIALSORT_OK;
}

dialsort_status launch_fill(const uint32_t* H, uint32_t* out, uint32_t lo, char* base, const Layout& L,
                            hipStream_t s, const uint32_t* lut = nullptr) {
  Ctl* ctl = (Ctl*)base;
  const FillItem* items = (const FillItem*)(base + L.off_items);
  const FillRun* runs = (const FillRun*)(base + L.off_runs);
  const uint32_t rcap = (uint32_t)std::min<uint64_t>(L.run_cap, 0xFFFFFFF0ull);
  if (L.limit == 0) return DIALSORT_OK;
  // one resident round of workgroups (8 per CU at 256 threads), or fewer
  const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(L.item_cap, FILL_NT / WAVE), 256 * 8);
  const uint32_t icap = (uint32_t)std::min<uint64_t>(L.item_cap, 0xFFFFFFF0ull);
  // an output larger than the L2 caches together is streamed past them: its
  // dirty lines then do not drain into the next kernel's HBM traffic
  const bool nts = L.limit * 4 >= FILL_NTS_BYTES;
  if (lut) {
    if (aligned16(out) && nts)
      DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, true, true, true>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, 0u, lut, runs, rcap);
    else if (aligned16(out))
      DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, true, true>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, 0u, lut, runs, rcap);
    else
      DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, false, true>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, 0u, lut, runs, rcap);
  } else if (aligned16(out) && nts) {
    DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, true, false, true>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, lo, nullptr, runs, rcap);
  } else if (aligned16(out)) {
    DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, true>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, lo, nullptr, runs, rcap);
  } else {
    DS_LAUNCH((k_fill<FILL_NT, FILL_CL2, false>), dim3(grid), dim3(FILL_NT), s, H, out, ctl, items, icap, lo, nullptr, runs, rcap);
  }
  return DIALSORT_OK;
}

// Accumulating ingestion: the keys' histogram goes to a scratch row T of the
// workspace (after the ingestion's own workspace), then k_accumulate adds T
// into H, reporting a bin that passes 2^32 - 1 as ST_OVERFLOW.
size_t accumulate_ws_off(uint64_t n, uint64_t U) { return align_up(plan(n, U, DIALSORT_MODE_HISTOGRAM).bytes, ALIGN); }
size_t accumulate_ws_bytes(uint64_t n, uint64_t U) { return accumulate_ws_off(n, U) + align_up(U * 4, ALIGN) + ALIGN; }

__global__ void k_accumulate(uint32_t* __restrict__ H, const uint32_t* __restrict__ T, uint64_t U, Ctl* ctl) {
  bool wrapped = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < U; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t a = H[i], s = a + T[i];
    wrapped |= s < a;
    H[i] = s;
  }
  if (__any(wrapped) && lane_id() == 0) set_status(ctl, ST_OVERFLOW);
}

dialsort_status check_common(uint64_t U, const void* ws, size_t ws_bytes, size_t need) {
  if (U == 0 || U > U_MAX) return DIALSORT_EINVAL;
  if (!ws || ws_bytes < need) return DIALSORT_EWORKSPACE;
  return DIALSORT_OK;
}

// A fresh launch epoch for k_sort_lds: a process-wide sequence from a random
// start, never 0.
uint64_t next_epoch() {
  static std::atomic<uint64_t> seq{[] {
    uint64_t r = 0;
    try {
      std::random_device rd;
      r = ((uint64_t)rd() << 32) | rd();
    } catch (...) {
      r = (uint64_t)(uintptr_t)&r;  // no entropy source: the clock below still varies
    }
    const uint64_t t = (uint64_t)std::chrono::steady_clock::now().time_since_epoch().count();
    return r ^ (t * 0x9E3779B97F4A7C15ull);
  }()};
  uint64_t e;
  do { e = seq.fetch_add(1, std::memory_order_relaxed); } while (e == 0);
  return e;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// The one-launch sort, outside graph capture.
bool use_fused(const Layout& L, hipStream_t s) { return L.fused && !capturing(s); }

dialsort_status launch_sort_fused(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t* H, uint32_t* out,
                                  char* base, const Layout& L, const FillCfg& fc, hipStream_t s) {
  const bool ka = aligned16(keys);
  uint32_t* rows = (uint32_t*)(base + L.off_rows);
  uint32_t* pre = (uint32_t*)(base + L.off_pre);
  uint64_t* flags = (uint64_t*)(base + L.off_flags);
  const uint64_t epoch = next_epoch();
  const dim3 grid(L.G + L.NS);
#define DS_FUSED(CAP, PACKED, KA)                                                                              \
  DS_LAUNCH((k_sort_lds<FUSED_NT, CAP, PACKED, 8, KA, 4>), grid, dim3(FUSED_NT), s, keys, n, L.per,            \
            (uint32_t)(U - 1), (uint32_t)U, L.G, L.NS, rows, L.row_stride, pre, (Ctl*)base, flags, epoch, H, out, \
            fc)
  switch (L.kind) {
    case K_LDS32S: if (ka) DS_FUSED(4096, false, true); else DS_FUSED(4096, false, false); break;
    case K_LDS32: if (ka) DS_FUSED(32768, false, true); else DS_FUSED(32768, false, false); break;
    case K_LDS16: if (ka) DS_FUSED(32768, true, true); else DS_FUSED(32768, true, false); break;
    default: return DIALSORT_EINVAL;
  }
#undef DS_FUSED
  return DIALSORT_OK;
}

// histogram or sort, after argument checks
dialsort_status run_sort(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t lo, uint32_t* H, uint32_t* out, void* ws,
                         int mode, hipStream_t s, const uint32_t* lut = nullptr) {
  const Layout L = plan(n, U, mode);
  char* base = ws_base(ws);
  const bool zeroH = L.kind == K_EMPTY || L.kind == K_GLOBAL;
  if (use_fused(L, s)) {
    FillCfg fc;
    fc.lo = lo;
    fc.lut = lut;
    fc.limit = n;
    fc.oal = aligned16(out);
    fc.nts = fc.oal && n * 4 >= FILL_NTS_BYTES;
    return launch_sort_fused(keys, n, U, H, out, base, L, fc, s);
  }
  if (!fold_init(L)) DS_TRY(launch_init(base, L, H, zeroH ? U : 0, s));
  DS_TRY(launch_ingest(keys, n, U, lo, H, base, L, s));
  const uint32_t* rows = L.rows_in_ws ? (const uint32_t*)(base + L.off_rows) : H;
  const uint32_t nrows = L.rows_in_ws ? L.G : 1;
  if (mode == DIALSORT_MODE_HISTOGRAM) {
    if (L.rows_in_ws) DS_TRY(launch_scan(rows, nrows, L.row_stride, H, U, base, L, false, 0, s));
    return DIALSORT_OK;
  }
  if (L.direct) {
    FillCfg fc;
    fc.lo = lo;
    fc.lut = lut;
    fc.limit = n;
    fc.oal = aligned16(out);
    fc.nts = fc.oal && n * 4 >= FILL_NTS_BYTES;
    return launch_scan(rows, nrows, L.rows_in_ws ? L.row_stride : 0, L.rows_in_ws ? H : nullptr, U, base, L, true, 0,
                       s, out, fc);
  }
  if (L.kind != K_PART)
    DS_TRY(launch_scan(rows, nrows, L.rows_in_ws ? L.row_stride : 0, L.rows_in_ws ? H : nullptr, U, base, L,
                       true, 0, s));
  DS_TRY(launch_fill(H, out, lo, base, L, s, lut));
  return DIALSORT_OK;
}

__global__ void k_or_status(Ctl* dst, const Ctl* src) {
  if (threadIdx.x == 0 && src->status) atomicOr(&dst->status, src->status);
}

}  // namespace

namespace dsh {

dialsort_status check_desc(const dialsort_desc& d) {
  if (d.U == 0 || d.U > U_MAX || !d.H || (d.n && (!d.keys || !d.out))) return DIALSORT_EINVAL;
  if (!aligned4(d.keys) || !aligned4(d.H) || !aligned4(d.out)) return DIALSORT_EINVAL;
  if (d.n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(d.keys, d.n * 4, d.H, d.U * 4) || overlap(d.out, d.n * 4, d.H, d.U * 4)) return DIALSORT_EINVAL;
  if (d.out != d.keys && overlap(d.keys, d.n * 4, d.out, d.n * 4)) return DIALSORT_EINVAL;
  return DIALSORT_OK;
}

size_t loop_workspace_bytes(const dialsort_desc* d, uint32_t count) {
  size_t mx = 0;
  for (uint32_t i = 0; i < count; ++i) {
    if (d[i].U == 0 || d[i].U > U_MAX) return 0;
    mx = std::max(mx, plan(d[i].n, d[i].U, DIALSORT_MODE_SORT).bytes);
  }
  return 2 * ALIGN + mx;
}

dialsort_status loop_run(const dialsort_desc* d, uint32_t count, void* ws, size_t ws_bytes, hipStream_t s) {
  if (count && !d) return DIALSORT_EINVAL;
  for (uint32_t i = 0; i < count; ++i) DS_TRY(check_desc(d[i]));
  if (!ws || ws_bytes < loop_workspace_bytes(d, count)) return DIALSORT_EWORKSPACE;
  char* base = ws_base(ws);
  Layout L0;
  L0.scan = false;
  DS_TRY(launch_init(base, L0, nullptr, 0, s));
  char* sub = base + ALIGN;
  for (uint32_t i = 0; i < count; ++i) {
    DS_TRY(run_sort(d[i].keys, d[i].n, d[i].U, 0, d[i].H, d[i].out, sub, DIALSORT_MODE_SORT, s));
    DS_LAUNCH(k_or_status, dim3(1), dim3(64), s, (Ctl*)base, (const Ctl*)sub);
  }
  return DIALSORT_OK;
}

}  // namespace dsh

extern "C" {

size_t dialsort_workspace_bytes(uint64_t n, uint64_t U, int mode) {
  if (U == 0 || U > U_MAX) return 0;
  if (mode == DIALSORT_MODE_ACCUMULATE) return accumulate_ws_bytes(n, U);
  return plan(n, U, mode).bytes;
}

dialsort_status dialsort_histogram(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t* H, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && !keys)) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(n, U, DIALSORT_MODE_HISTOGRAM)));
  CallScope scope(stream);
  return run_sort(keys, n, U, 0, H, nullptr, ws, DIALSORT_MODE_HISTOGRAM, stream);
}

dialsort_status dialsort_histogram_accumulate(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t* H, void* ws,
                                              size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && !keys)) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, accumulate_ws_bytes(n, U)));
  CallScope scope(stream);
  char* base = ws_base(ws);
  uint32_t* T = (uint32_t*)(base + accumulate_ws_off(n, U));
  DS_TRY(run_sort(keys, n, U, 0, T, nullptr, ws, DIALSORT_MODE_HISTOGRAM, stream));
  const uint32_t grid = (uint32_t)std::min<uint64_t>(cdiv(U, 256), 256 * 8);
  DS_LAUNCH(k_accumulate, dim3(grid), dim3(256), stream, H, T, U, (Ctl*)base);
  return DIALSORT_OK;
}

dialsort_status dialsort_histogram_offset(const uint32_t* keys, uint64_t n, uint32_t lo, uint64_t U, uint32_t* H,
                                          void* ws, size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && !keys)) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(n, U, DIALSORT_MODE_HISTOGRAM)));
  CallScope scope(stream);
  return run_sort(keys, n, U, lo, H, nullptr, ws, DIALSORT_MODE_HISTOGRAM, stream);
}

dialsort_status dialsort_sort_offset(const uint32_t* keys, uint64_t n, uint32_t lo, uint64_t U, uint32_t* H,
                                     uint32_t* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && (!keys || !out))) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H) || !aligned4(out)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4) || overlap(out, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  if (out != keys && overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(n, U, DIALSORT_MODE_SORT)));
  CallScope scope(stream);
  return run_sort(keys, n, U, lo, H, out, ws, DIALSORT_MODE_SORT, stream);
}

dialsort_status dialsort_sort_lut(const uint32_t* keys, uint64_t n, uint64_t U, const uint32_t* lut, uint32_t* H,
                                  uint32_t* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || !lut || (n && (!keys || !out))) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H) || !aligned4(out) || !aligned4(lut)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4) || overlap(out, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  if (overlap(lut, U * 4, H, U * 4) || overlap(lut, U * 4, out, n * 4)) return DIALSORT_EINVAL;
  if (out != keys && overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(n, U, DIALSORT_MODE_SORT)));
  CallScope scope(stream);
  return run_sort(keys, n, U, 0, H, out, ws, DIALSORT_MODE_SORT, stream, lut);
}

dialsort_status dialsort_sort(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t* H, uint32_t* out, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && (!keys || !out))) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H) || !aligned4(out)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4) || overlap(out, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  if (out != keys && overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(n, U, DIALSORT_MODE_SORT)));
  CallScope scope(stream);
  return run_sort(keys, n, U, 0, H, out, ws, DIALSORT_MODE_SORT, stream);
}

dialsort_status dialsort_reconstruct(const uint32_t* H, uint64_t U, uint32_t* out, uint64_t out_cap, void* ws,
                                     size_t ws_bytes, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (out_cap && !out)) return DIALSORT_EINVAL;
  if (!aligned4(H) || !aligned4(out)) return DIALSORT_EINVAL;
  if (out_cap > LB_VAL - 1) return DIALSORT_EINVAL;
  if (out_cap && overlap(out, out_cap * 4, H, U * 4)) return DIALSORT_EINVAL;
  DS_TRY(check_common(U, ws, ws_bytes, dialsort_workspace_bytes(out_cap, U, DIALSORT_MODE_RECONSTRUCT)));
  const Layout L = plan(out_cap, U, DIALSORT_MODE_RECONSTRUCT);
  char* base = ws_base(ws);
  CallScope scope(stream);
  DS_TRY(launch_init(base, L, nullptr, 0, stream));
  DS_TRY(launch_scan(H, 1, 0, nullptr, U, base, L, true, 1, stream));
  DS_TRY(launch_fill(H, out, 0, base, L, stream));
  return DIALSORT_OK;
}

// Tumbling windows: window w is ingested on `ingest` into H + (w mod 2) U and
// projected on `project` while window w + 1 is ingested into the other
// histogram.  Each histogram has its own sub-workspace, used in turn by its
// window's ingestion and projection; the combined status lives at the front.
static size_t windows_sub_bytes(uint64_t wn, uint64_t U) {
  return align_up(std::max(plan(wn, U, DIALSORT_MODE_HISTOGRAM).bytes, plan(wn, U, DIALSORT_MODE_RECONSTRUCT).bytes),
                  ALIGN);
}

size_t dialsort_windows_workspace_bytes(uint64_t window_n, uint64_t U) {
  if (U == 0 || U > U_MAX || window_n > N_MAX) return 0;
  return 2 * ALIGN + 2 * windows_sub_bytes(window_n, U);
}

dialsort_status dialsort_sort_windows(const uint32_t* keys, uint64_t window_n, uint32_t count, uint64_t U,
                                      uint32_t* H, uint32_t* out, void* ws, size_t ws_bytes, hipStream_t ingest,
                                      hipStream_t project) {
  const uint64_t n = window_n * count;
  if (U == 0 || U > U_MAX || !H || (n && (!keys || !out))) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H) || !aligned4(out)) return DIALSORT_EINVAL;
  if (window_n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, 2 * U * 4) || overlap(out, n * 4, H, 2 * U * 4)) return DIALSORT_EINVAL;
  if (overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  if (!ws || ws_bytes < dialsort_windows_workspace_bytes(window_n, U)) return DIALSORT_EWORKSPACE;
  char* base = ws_base(ws);
  const size_t sub_bytes = windows_sub_bytes(window_n, U);
  char* sub[2] = {base + ALIGN, base + ALIGN + sub_bytes};
  CallScope scope(project);
  Layout L0;
  L0.scan = false;
  DS_TRY(launch_init(base, L0, nullptr, 0, project));
  if (count == 0) return DIALSORT_OK;
  // ingested[0], ingested[1], projected[0], projected[1], and the point on
  // `project` where this call starts: the first two ingestions reuse the
  // sub-workspaces and histograms that work enqueued earlier on `project` (a
  // previous call's last projections) may still read
  hipEvent_t ev[5] = {};
  dialsort_status st = DIALSORT_OK;
  for (int i = 0; i < 5 && st == DIALSORT_OK; ++i) {
    const hipError_t e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      g_last_hip_error = (int)e;
      st = DIALSORT_EHIP;
    }
  }
  const Layout LR = plan(window_n, U, DIALSORT_MODE_RECONSTRUCT);
  auto run = [&]() -> dialsort_status {
    DS_HIP(hipEventRecord(ev[4], project));
    DS_HIP(hipStreamWaitEvent(ingest, ev[4], 0));
    for (uint32_t w = 0; w < count; ++w) {
      const int b = (int)(w & 1u);
      uint32_t* Hb = H + (uint64_t)b * U;
      char* sb = sub[b];
      // window w - 2 has been projected out of this histogram and workspace
      if (w >= 2) DS_HIP(hipStreamWaitEvent(ingest, ev[2 + b], 0));
      DS_TRY(run_sort(keys + (uint64_t)w * window_n, window_n, U, 0, Hb, nullptr, sb, DIALSORT_MODE_HISTOGRAM,
                      ingest));
      DS_HIP(hipEventRecord(ev[b], ingest));
      DS_HIP(hipStreamWaitEvent(project, ev[b], 0));
      // the ingestion's status, before the projection clears the workspace
      DS_LAUNCH(k_or_status, dim3(1), dim3(64), project, (Ctl*)base, (const Ctl*)sb);
      DS_TRY(launch_init(sb, LR, nullptr, 0, project));
      DS_TRY(launch_scan(Hb, 1, 0, nullptr, U, sb, LR, true, 1, project));
      DS_TRY(launch_fill(Hb, out + (uint64_t)w * window_n, 0, sb, LR, project));
      DS_LAUNCH(k_or_status, dim3(1), dim3(64), project, (Ctl*)base, (const Ctl*)sb);
      DS_HIP(hipEventRecord(ev[2 + b], project));
    }
    // the last ingestion is also ordered before everything that follows on project
    return DIALSORT_OK;
  };
  if (st == DIALSORT_OK) st = run();
  for (int i = 0; i < 5; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  return st;
}

dialsort_status dialsort_set_launch_events(hipEvent_t* events, uint32_t cap, uint32_t* count) {
  if (events && cap < 2) return DIALSORT_EINVAL;
  g_log.ev = events;
  g_log.cap = events ? cap : 0;
  g_log.count = events ? count : nullptr;
  if (g_log.names.size() < std::max<uint32_t>(g_log.cap, 64)) g_log.names.resize(std::max<uint32_t>(g_log.cap, 64));
  return DIALSORT_OK;
}

const char* dialsort_launch_name(uint32_t i) {
  return i < g_log.n && i < g_log.names.size() ? g_log.names[i] : nullptr;
}

dialsort_status dialsort_status_sync(const void* ws, hipStream_t stream) {
  if (!ws) return DIALSORT_EINVAL;
  uint32_t st = 0;
  const char* base = ws_base(const_cast<void*>(ws));
  hipError_t e = hipMemcpyAsync(&st, base + offsetof(Ctl, status), 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    return DIALSORT_EHIP;
  }
  if (st & ST_RANGE) return DIALSORT_ERANGE;
  if (st & ST_OVERFLOW) return DIALSORT_EOVERFLOW;
  if (st) return DIALSORT_EHIP;
  return DIALSORT_OK;
}

dialsort_status dialsort_result_total(const void* ws, hipStream_t stream, uint64_t* total) {
  if (!ws || !total) return DIALSORT_EINVAL;
  const char* base = ws_base(const_cast<void*>(ws));
  hipError_t e = hipMemcpyAsync(total, base + offsetof(Ctl, total), 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    return DIALSORT_EHIP;
  }
  return DIALSORT_OK;
}

}  // extern "C"

// ---- the allocation-free sort -----------------------------------------------
// dialsort_sort_noalloc runs dialsort_sort's kernels with their workspace in
// `scratch`, a device array of this library: each device holds its own copy
// from module load until the process ends.  In host code the array's name is
// only a stand-in; its device address comes from hipGetSymbolAddress, taken
// once per device (with that device current) and kept.
namespace {

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal

dialsort_status scratch_of_current_device(void** p) {
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    DS_HIP(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
    if (!q) return DIALSORT_EHIP;
    g_scratch_ptr[dev] = q;
  }
  *p = g_scratch_ptr[dev];
  return DIALSORT_OK;
}

__global__ void k_copy_status(uint32_t* dst, const Ctl* src) {
  if (threadIdx.x == 0) *dst = src->status;
}

}  // namespace

extern "C" {

dialsort_status dialsort_sort_noalloc(const uint32_t* keys, uint64_t n, uint64_t U, uint32_t* H, uint32_t* out,
                                      uint32_t* status, hipStream_t stream) {
  if (U == 0 || U > U_MAX || !H || (n && (!keys || !out))) return DIALSORT_EINVAL;
  if (!aligned4(keys) || !aligned4(H) || !aligned4(out) || !aligned4(status)) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  if (overlap(keys, n * 4, H, U * 4) || overlap(out, n * 4, H, U * 4)) return DIALSORT_EINVAL;
  if (out != keys && overlap(keys, n * 4, out, n * 4)) return DIALSORT_EINVAL;
  if (status && (overlap(status, 4, keys, n * 4) || overlap(status, 4, H, U * 4) || overlap(status, 4, out, n * 4)))
    return DIALSORT_EINVAL;
  if (dialsort_workspace_bytes(n, U, DIALSORT_MODE_SORT) > NOALLOC_BYTES) return DIALSORT_EWORKSPACE;
  void* ws = nullptr;
  DS_TRY(scratch_of_current_device(&ws));
  CallScope scope(stream);
  DS_TRY(run_sort(keys, n, U, 0, H, out, ws, DIALSORT_MODE_SORT, stream));
  if (status) DS_LAUNCH(k_copy_status, dim3(1), dim3(64), stream, status, (const Ctl*)ws_base(ws));
  return DIALSORT_OK;
}

const char* dialsort_strerror(dialsort_status status) {
  switch (status) {
    case DIALSORT_OK: return "ok";
    case DIALSORT_EINVAL: return "invalid argument";
    case DIALSORT_ERANGE: return "key outside [0, U)";
    case DIALSORT_EOVERFLOW: return "count overflow (n > 2^32-1 or sum(H) > out_cap)";
    case DIALSORT_EWORKSPACE: return "workspace missing or too small";
    case DIALSORT_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

int dialsort_last_hip_error(void) { return g_last_hip_error; }

}  // extern "C"
