// libdialsort, batched entry points: many independent arrays sorted by one
// persistent launch (csrc/batch.hpp), its host-side planner, the autotuner that
// chooses block size, U-partition width and privatization depth, and the
// per-array launch sequences used as the plain baseline and as the fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/dialsort.h"
#include "batch.hpp"
#include "batch_host.hpp"
#include "host_common.hpp"

using namespace ds;
using namespace dsh;

namespace dsb {

constexpr uint32_t UNIT_KEYS = 1u << 19;  // target keys per A or B unit
constexpr uint32_t FILL_PER = 64;         // item slots per fill unit (shared by its waves)
constexpr uint64_t CLASS_MIN_COST = 1ull << 22;  // keys plus bins of the first size class, at least
constexpr uint64_t CLASS_GROWTH = 3;             // a class closes at this many times the cost before it
constexpr uint64_t BT_PACKED_CHUNK_MAX = 1ull << 22;
constexpr uint64_t LATE_FILL_NUM = 1, LATE_FILL_DEN = 4;  // classes ending past this share of the cost
                                                           // fill in k_batch_fill
constexpr int FILL_K_NT = 256;                             // k_batch_fill workgroup

bool cfg_valid(const dialsort_batch_config& c) {
  const bool nt = c.block == 512 || c.block == 1024;
  const bool w = c.log2_width >= 14 && c.log2_width <= 16;
  const bool ch = c.chunk_keys >= (1ull << 16) && c.chunk_keys <= (1ull << 22) &&
                  (c.chunk_keys & (c.chunk_keys - 1)) == 0;
  return nt && w && ch;
}

Cfg to_cfg(const dialsort_batch_config& c) {
  Cfg r;
  r.nt = c.block;
  r.log2w = c.log2_width;
  r.chunk = c.chunk_keys;
  return r;
}

dialsort_batch_config from_cfg(const Cfg& c) {
  dialsort_batch_config r;
  r.block = c.nt;
  r.log2_width = c.log2w;
  r.chunk_keys = c.chunk;
  return r;
}

// The arrays the fused launch takes: U <= BT_BMAX * W, 16-byte aligned keys, H
// and output (the other arrays go through the per-array launch sequences).
bool fused_ok(const dialsort_desc& d, const Cfg& c) {
  if (d.U > ((uint64_t)BT_BMAX << c.log2w)) return false;
  if (!aligned16(d.H)) return false;
  if (d.n && (!aligned16(d.keys) || !aligned16(d.out))) return false;
  return true;
}

// Lay out the batch in a workspace based at `base` (null: sizes only):
// [Ctl][arrays][states][units][per-array rows / staging / segments / items].
void plan_batch(const dialsort_desc* d, uint32_t count, const Cfg& cfg, char* base, Planned& P) {
  const uint64_t W = 1ull << cfg.log2w;
  const uint64_t C = 1ull << BT_CL2;
  const uint64_t piece = std::min<uint64_t>(W, 1ull << 15);
  P.arr.assign(count, BArray{});
  P.units.clear();
  // shapes
  for (uint32_t i = 0; i < count; ++i) {
    BArray& A = P.arr[i];
    A.keys = d[i].keys;
    A.H = d[i].H;
    A.out = d[i].out;
    A.n = d[i].n;
    A.U = d[i].U;
    const uint64_t n = A.n, U = A.U;
    if (n == 0) {
      A.kind = BA_EMPTY;
      A.na = 0;
      A.nb = 1;
      A.item_cap = 0;
    } else if (U <= W) {
      A.kind = BA_LDS;
      const uint64_t chunk = std::min<uint64_t>(cfg.chunk, BT_PACKED_CHUNK_MAX);
      A.per = std::min<uint64_t>(chunk, align_up(n, 4));
      A.na = (uint32_t)cdiv(n, A.per);
      A.row_stride = A.na == 1 ? 0 : align_up(U, 64);
      A.nb = 1;
      // one item per chunk of C positions plus one per projection tile and per
      // piece of the universe, where a span boundary splits a chunk
      A.item_cap = (uint32_t)(cdiv(n, C) + cdiv(U, PT_BINS) + 2 * cdiv(U, piece) + 2);
    } else {
      A.kind = BA_PART;
      A.B = (uint32_t)cdiv(U, W);
      A.na = (uint32_t)cdiv(n, BT_TK);
      A.bstride = (uint32_t)align_up(A.B + 1, 8);
      A.nb = A.B;
      // every projection tile is one span; every bucket one piece (two for a
      // heavy bucket counted in halves)
      A.item_cap = (uint32_t)(cdiv(n, C) + cdiv(U, PT_BINS) + 2ull * A.B + 2);
    }
    A.nf = A.item_cap ? (uint32_t)cdiv(A.item_cap, FILL_PER) : 0;
  }
  // Units in size classes: arrays sorted by cost (keys plus bins), cut into
  // classes whose cost grows geometrically (a class closes once it holds as
  // much as all the classes before it, times CLASS_GROWTH), and each class
  // laid out phase by phase (all its ingestion units, then its counting
  // units, then its fill units), larger arrays first inside a phase.  Small
  // arrays then complete early, while every phase of a class still runs wide.
  // Without classes (cfg.classes false) the whole batch is one class.  A unit
  // waits only for units of its own array with smaller tickets.
  std::vector<uint32_t> order(count);
  std::iota(order.begin(), order.end(), 0u);
  auto cost = [&](uint32_t i) { return d[i].n + d[i].U; };
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost(a) < cost(b); });
  auto add = [&](uint32_t a, uint32_t type, uint32_t first, uint32_t cnt) {
    BUnit u;
    u.array = a; u.type = type; u.first = first; u.count = cnt;
    P.units.push_back(u);
  };
  std::vector<BUnit> late;  // fill units of the late classes, listed last
  auto emit_class = [&](std::vector<uint32_t> cls, bool late_fill) {
    std::stable_sort(cls.begin(), cls.end(), [&](uint32_t a, uint32_t b) { return d[a].n > d[b].n; });
    for (uint32_t i : cls) {
      const BArray& A = P.arr[i];
      if (A.kind == BA_LDS) {
        const uint32_t g = (uint32_t)std::max<uint64_t>(1, UNIT_KEYS / A.per);
        for (uint32_t c = 0; c < A.na; c += g) add(i, UT_HIST, c, std::min(g, A.na - c));
      } else if (A.kind == BA_PART) {
        const uint32_t g = UNIT_KEYS / BT_TK;
        for (uint32_t t = 0; t < A.na; t += g) add(i, UT_PART, t, std::min(g, A.na - t));
      }
    }
    for (uint32_t i : cls) {
      const BArray& A = P.arr[i];
      if (A.kind == BA_PART) {
        // a bucket costs its keys plus a fixed sweep of its W bins
        const uint64_t bc = A.n / A.B + W / 4;
        const uint32_t g = (uint32_t)std::max<uint64_t>(1, UNIT_KEYS / bc);
        for (uint32_t b = 0; b < A.B; b += g) add(i, UT_BUCKET, b, std::min(g, A.B - b));
      } else {
        add(i, UT_ROWS, 0, 1);
      }
    }
    for (uint32_t i : cls) {
      const BArray& A = P.arr[i];
      for (uint32_t f = 0; f < A.nf; ++f) {
        add(i, UT_FILL, f, A.nf);
        if (late_fill) {
          late.push_back(P.units.back());
          P.units.pop_back();
        }
      }
    }
  };
  // a class whose cost ends past LATE_FILL of the batch's leaves its fills to
  // k_batch_fill (a single class always does)
  uint64_t all_cost = 0;
  for (uint32_t i = 0; i < count; ++i) all_cost += cost(i);
  auto late_end = [&](uint64_t end_cost) { return end_cost * LATE_FILL_DEN > all_cost * LATE_FILL_NUM; };
  std::vector<uint32_t> cls;
  uint64_t done_cost = 0, cls_cost = 0;
  for (uint32_t i : order) {
    cls.push_back(i);
    cls_cost += cost(i);
    if (cfg.classes && cls_cost >= std::max<uint64_t>(CLASS_MIN_COST, CLASS_GROWTH * done_cost)) {
      emit_class(cls, late_end(done_cost + cls_cost));
      done_cost += cls_cost;
      cls_cost = 0;
      cls.clear();
    }
  }
  if (!cls.empty()) emit_class(cls, true);
  P.fill_units = (uint32_t)late.size();
  P.units.insert(P.units.end(), late.begin(), late.end());
  // offsets
  size_t off = ALIGN;  // Ctl
  P.off_arrays = off;
  off = align_up(off + (size_t)count * sizeof(BArray), ALIGN);
  P.off_states = off;
  off = align_up(off + (size_t)count * sizeof(BState), ALIGN);
  P.off_units = off;
  off = align_up(off + P.units.size() * sizeof(BUnit), ALIGN);
  auto at = [&](size_t o) -> char* { return base ? base + o : nullptr; };
  for (uint32_t i = 0; i < count; ++i) {
    BArray& A = P.arr[i];
    if (A.kind == BA_LDS) {
      if (A.na == 1) {
        A.rows = A.H;
      } else {
        A.rows = (uint32_t*)at(off);
        off = align_up(off + (size_t)A.na * A.row_stride * 4, ALIGN);
      }
    } else if (A.kind == BA_PART) {
      A.staging = (uint16_t*)at(off);
      off = align_up(off + ((size_t)A.na * BT_TK + 16) * 2, ALIGN);  // whole tiles
      A.seg = (uint16_t*)at(off);
      off = align_up(off + (size_t)A.na * A.bstride * 2, ALIGN);
    }
    if (A.item_cap) {
      A.items = (FillItem*)at(off);
      off = align_up(off + (size_t)A.item_cap * sizeof(FillItem), ALIGN);
    }
  }
  P.bytes = off + ALIGN;  // slack for aligning the caller's pointer
}

// Candidate configurations of the autotuner.
std::vector<Cfg> candidates() {
  std::vector<Cfg> v;
  for (uint32_t nt : {512u, 1024u})
    for (uint32_t w : {14u, 15u, 16u})
      for (uint64_t ch : {1ull << 18, 1ull << 20, 1ull << 22}) {
        Cfg c;
        c.nt = nt; c.log2w = w; c.chunk = ch;
        v.push_back(c);
      }
  return v;
}

// Persistent grid of k_batch_fill: every workgroup the device holds at once,
// at most one per unit.  The occupancy is queried once per device.
std::mutex g_fill_occ_mu;
std::map<int, uint32_t> g_fill_occ;

uint32_t fill_grid(uint32_t units) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  uint32_t resident = 0;
  {
    std::lock_guard<std::mutex> lk(g_fill_occ_mu);
    auto it = g_fill_occ.find(dev);
    if (it != g_fill_occ.end()) {
      resident = it->second;
    } else {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_fill<FILL_K_NT>, FILL_K_NT, 0) != hipSuccess)
        nb = 1;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 1;
      resident = (uint32_t)(std::max(nb, 1) * std::max(cus, 1));
      g_fill_occ[dev] = resident;
    }
  }
  return std::max<uint32_t>(1, std::min(resident, units));
}

template <int NT, int LOG2W>
dialsort_status launch_fused_t(const dialsort_batch_plan& p, hipStream_t s) {
  char* base = ws_base(p.ws);
  const size_t off_arrays = ALIGN;
  const size_t off_states = align_up(off_arrays + (size_t)p.count * sizeof(BArray), ALIGN);
  const size_t off_units = (size_t)p.units_offset;
  const uint32_t ig = (uint32_t)cdiv(std::max<uint64_t>(64, (uint64_t)p.count * 8), 256);
  DS_LAUNCH(k_batch_init, dim3(std::min<uint32_t>(ig, 1024)), dim3(256), s, (Ctl*)base, (BState*)(base + off_states),
            p.count);
  const uint32_t nmain = p.units - p.fill_units;
  if (nmain)
    DS_LAUNCH((k_batch<NT, LOG2W>), dim3(p.grid), dim3(NT), s, (const BArray*)(base + off_arrays),
              (BState*)(base + off_states), (const BUnit*)(base + off_units), nmain, (Ctl*)base);
  if (p.fill_units)
    DS_LAUNCH((k_batch_fill<FILL_K_NT>), dim3(fill_grid(p.fill_units)), dim3(FILL_K_NT), s,
              (const BArray*)(base + off_arrays), (BState*)(base + off_states),
              (const BUnit*)(base + off_units) + nmain, p.fill_units, (Ctl*)base);
  return DIALSORT_OK;
}

dialsort_status launch_fused(const dialsort_batch_plan& p, hipStream_t s) {
  const uint32_t nt = p.config.block, w = p.config.log2_width;
  if (nt == 512 && w == 14) return launch_fused_t<512, 14>(p, s);
  if (nt == 512 && w == 15) return launch_fused_t<512, 15>(p, s);
  if (nt == 512 && w == 16) return launch_fused_t<512, 16>(p, s);
  if (nt == 1024 && w == 14) return launch_fused_t<1024, 14>(p, s);
  if (nt == 1024 && w == 15) return launch_fused_t<1024, 15>(p, s);
  if (nt == 1024 && w == 16) return launch_fused_t<1024, 16>(p, s);
  return DIALSORT_EINVAL;
}

template <int NT, int LOG2W>
int occupancy_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<NT, LOG2W>, NT, 0) != hipSuccess) return 1;
  return std::max(nb, 1);
}

// Resident workgroups per CU of the fused kernel, per configuration.
int occupancy_query(const Cfg& c) {
  if (c.nt == 512 && c.log2w == 14) return occupancy_t<512, 14>();
  if (c.nt == 512 && c.log2w == 15) return occupancy_t<512, 15>();
  if (c.nt == 512 && c.log2w == 16) return occupancy_t<512, 16>();
  if (c.nt == 1024 && c.log2w == 14) return occupancy_t<1024, 14>();
  if (c.nt == 1024 && c.log2w == 15) return occupancy_t<1024, 15>();
  return occupancy_t<1024, 16>();
}

std::mutex g_occ_mu;
std::map<std::pair<int, uint32_t>, int> g_occ;

int occupancy(const Cfg& c) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint32_t key = c.nt * 32u + c.log2w;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto it = g_occ.find({dev, key});
  if (it != g_occ.end()) return it->second;
  const int v = occupancy_query(c);
  g_occ[{dev, key}] = v;
  return v;
}

// Autotune cache: per device, batch shape -> best configuration.
std::mutex g_tune_mu;
std::map<std::pair<int, uint64_t>, Cfg> g_tuned;

uint64_t batch_signature(const dialsort_desc* d, uint32_t count) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t x) {
    for (int i = 0; i < 8; ++i) {
      h ^= (x >> (8 * i)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  mix(count);
  for (uint32_t i = 0; i < count; ++i) {
    mix(d[i].n);
    mix(d[i].U);
  }
  return h;
}

Cfg default_cfg(const dialsort_desc* d, uint32_t count) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find({dev, batch_signature(d, count)});
  if (it != g_tuned.end()) return it->second;
  return Cfg{};
}

size_t table_bytes(const Planned& P) { return P.off_units + P.units.size() * sizeof(BUnit) - P.off_arrays; }

void write_tables(const Planned& P, char* host) {
  std::memset(host, 0, table_bytes(P));
  std::memcpy(host, P.arr.data(), P.arr.size() * sizeof(BArray));
  std::memcpy(host + (P.off_units - P.off_arrays), P.units.data(), P.units.size() * sizeof(BUnit));
}

dialsort_status make_plan(const Planned& P, uint32_t count, const Cfg& cfg, void* ws, size_t ws_bytes,
                          dialsort_batch_plan* plan) {
  int dev = 0, cus = 0;
  DS_HIP(hipGetDevice(&dev));
  DS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const uint64_t resident = (uint64_t)occupancy(cfg) * (uint64_t)std::max(cus, 1);
  std::memset(plan, 0, sizeof(*plan));
  plan->config = from_cfg(cfg);
  plan->count = count;
  plan->units = (uint32_t)P.units.size();
  plan->fill_units = P.fill_units;
  plan->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(resident, P.units.size() - P.fill_units));
  if (P.fill_units) (void)fill_grid(P.fill_units);  // the occupancy query happens here, not in a capture
  plan->units_offset = P.off_units;
  plan->ws = ws;
  plan->ws_bytes = ws_bytes;
  return DIALSORT_OK;
}

dialsort_status prepare(const dialsort_desc* d, uint32_t count, const Cfg& cfg, void* ws, size_t ws_bytes,
                        hipStream_t s, dialsort_batch_plan* plan) {
  if (count && !d) return DIALSORT_EINVAL;
  for (uint32_t i = 0; i < count; ++i) {
    DS_TRY(check_desc(d[i]));
    if (!fused_ok(d[i], cfg)) return DIALSORT_EINVAL;
  }
  if (!ws) return DIALSORT_EWORKSPACE;
  char* base = ws_base(ws);
  Planned P;
  plan_batch(d, count, cfg, base, P);
  if (ws_bytes < P.bytes) return DIALSORT_EWORKSPACE;
  if (P.units.size() >= 0xFFFFFFF0ull) return DIALSORT_EINVAL;
  // tables: arrays, states (cleared again by every launch), units
  std::vector<char> host(table_bytes(P));
  write_tables(P, host.data());
  DS_HIP(hipMemcpyAsync(base + P.off_arrays, host.data(), host.size(), hipMemcpyHostToDevice, s));
  DS_HIP(hipStreamSynchronize(s));
  return make_plan(P, count, cfg, ws, ws_bytes, plan);
}

size_t fused_workspace_bytes(const dialsort_desc* d, uint32_t count) {
  size_t mx = 0;
  for (const Cfg& c : candidates()) {
    bool ok = true;
    for (uint32_t i = 0; i < count && ok; ++i) ok = fused_ok(d[i], c);
    if (!ok) continue;
    Planned P;
    plan_batch(d, count, c, nullptr, P);
    mx = std::max(mx, P.bytes);
  }
  return mx;
}

}  // namespace dsb

using namespace dsb;

extern "C" {

size_t dialsort_batched_workspace_bytes(const dialsort_desc* descs, uint32_t count) {
  if (count && !descs) return 0;
  for (uint32_t i = 0; i < count; ++i)
    if (descs[i].U == 0 || descs[i].U > U_MAX) return 0;
  return std::max(loop_workspace_bytes(descs, count), fused_workspace_bytes(descs, count));
}

dialsort_status dialsort_batch_default_config(const dialsort_desc* descs, uint32_t count,
                                              dialsort_batch_config* config) {
  if (!config || (count && !descs)) return DIALSORT_EINVAL;
  *config = from_cfg(default_cfg(descs, count));
  return DIALSORT_OK;
}

dialsort_status dialsort_batch_prepare(const dialsort_desc* descs, uint32_t count,
                                       const dialsort_batch_config* config, void* ws, size_t ws_bytes,
                                       hipStream_t stream, dialsort_batch_plan* plan) {
  if (!plan) return DIALSORT_EINVAL;
  if (config && !cfg_valid(*config)) return DIALSORT_EINVAL;
  const Cfg cfg = config ? to_cfg(*config) : default_cfg(descs, count);
  return prepare(descs, count, cfg, ws, ws_bytes, stream, plan);
}

dialsort_status dialsort_batch_launch(const dialsort_batch_plan* plan, hipStream_t stream) {
  if (!plan || !plan->ws || !cfg_valid(plan->config)) return DIALSORT_EINVAL;
  CallScope scope(stream);
  return launch_fused(*plan, stream);
}

dialsort_status dialsort_sort_batched(const dialsort_desc* descs, uint32_t count, void* ws, size_t ws_bytes,
                                      hipStream_t stream) {
  if (count && !descs) return DIALSORT_EINVAL;
  for (uint32_t i = 0; i < count; ++i) DS_TRY(check_desc(descs[i]));
  if (!ws || ws_bytes < dialsort_batched_workspace_bytes(descs, count)) return DIALSORT_EWORKSPACE;
  const Cfg cfg = default_cfg(descs, count);
  bool ok = true;
  for (uint32_t i = 0; i < count && ok; ++i) ok = fused_ok(descs[i], cfg);
  CallScope scope(stream);
  if (!ok || count == 0) return loop_run(descs, count, ws, ws_bytes, stream);
  dialsort_batch_plan plan;
  DS_TRY(prepare(descs, count, cfg, ws, ws_bytes, stream, &plan));
  return launch_fused(plan, stream);
}

dialsort_status dialsort_sort_each(const dialsort_desc* descs, uint32_t count, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
  CallScope scope(stream);
  return loop_run(descs, count, ws, ws_bytes, stream);
}

dialsort_status dialsort_batch_autotune(const dialsort_desc* descs, uint32_t count, void* ws, size_t ws_bytes,
                                        hipStream_t stream, dialsort_batch_config* best) {
  if (!best || (count && !descs) || count == 0) return DIALSORT_EINVAL;
  for (uint32_t i = 0; i < count; ++i) DS_TRY(check_desc(descs[i]));
  hipEvent_t e0, e1;
  DS_HIP(hipEventCreate(&e0));
  DS_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  Cfg best_cfg;
  bool found = false;
  dialsort_status rc = DIALSORT_OK;
  for (const Cfg& c : candidates()) {
    bool ok = true;
    for (uint32_t i = 0; i < count && ok; ++i) ok = fused_ok(descs[i], c);
    if (!ok) continue;
    dialsort_batch_plan plan;
    rc = prepare(descs, count, c, ws, ws_bytes, stream, &plan);
    if (rc != DIALSORT_OK) break;
    float t = 1e30f;
    for (int rep = 0; rep < 3 && rc == DIALSORT_OK; ++rep) {
      hipError_t e = hipEventRecord(e0, stream);
      if (e == hipSuccess) rc = launch_fused(plan, stream);
      if (rc == DIALSORT_OK && e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        g_last_hip_error = (int)e;
        rc = DIALSORT_EHIP;
      }
      if (rep > 0) t = std::min(t, ms);  // the first run warms up
    }
    if (rc != DIALSORT_OK) break;
    if (t < best_ms) {
      best_ms = t;
      best_cfg = c;
      found = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DIALSORT_OK) return rc;
  if (!found) return DIALSORT_EINVAL;
  int dev = 0;
  DS_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[{dev, batch_signature(descs, count)}] = best_cfg;
  }
  *best = from_cfg(best_cfg);
  return DIALSORT_OK;
}

dialsort_status dialsort_batch_times(const dialsort_batch_plan* plan, hipStream_t stream, double* array_ms,
                                     uint32_t count, double* launch_ms, double* unit_ms) {
  if (!plan || !plan->ws || (count && !array_ms) || count > plan->count) return DIALSORT_EINVAL;
  char* base = ws_base(plan->ws);
  const size_t off_states = align_up(ALIGN + (size_t)plan->count * sizeof(BArray), ALIGN);
  std::vector<BState> st(count);
  Ctl ctl;
  DS_HIP(hipMemcpyAsync(&ctl, base, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
  if (count) DS_HIP(hipMemcpyAsync(st.data(), base + off_states, count * sizeof(BState), hipMemcpyDeviceToHost, stream));
  DS_HIP(hipStreamSynchronize(stream));
  int dev = 0, khz = 0;
  DS_HIP(hipGetDevice(&dev));
  DS_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  const double tick_ms = khz > 0 ? 1.0 / khz : 0.0;
  for (uint32_t i = 0; i < count; ++i)
    array_ms[i] = st[i].t_done >= ctl.total ? (double)(st[i].t_done - ctl.total) * tick_ms : 0.0;
  if (launch_ms) *launch_ms = ctl.limit >= ctl.total ? (double)(ctl.limit - ctl.total) * tick_ms : 0.0;
  if (unit_ms)
    for (int i = 0; i < 12; ++i) unit_ms[i] = (double)ctl.prof[i] * tick_ms;
  return DIALSORT_OK;
}

}  // extern "C"
