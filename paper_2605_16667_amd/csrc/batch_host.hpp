// Host side of the fused batched launch, shared by the batched entry points and
// the serving engine: configuration, the planner that lays a batch out in a
// workspace and lists its work units, the table upload format, and the launch.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/dialsort.h"
#include "batch.hpp"

namespace dsb {

struct Cfg {
  uint32_t nt = 1024, log2w = 16;
  uint64_t chunk = 1ull << 20;
  // lay the units out in size classes (small arrays complete early); off:
  // phase by phase over the whole batch, for callers that only wait for the
  // whole launch
  bool classes = true;
};

struct Planned {
  std::vector<ds::BArray> arr;
  std::vector<ds::BUnit> units;  // the fused kernel's units, then fill_units for k_batch_fill
  uint32_t fill_units = 0;
  size_t off_arrays = 0, off_states = 0, off_units = 0, bytes = 0;
};

bool cfg_valid(const dialsort_batch_config& c);
Cfg to_cfg(const dialsort_batch_config& c);
dialsort_batch_config from_cfg(const Cfg& c);

// Arrays the fused launch takes (U small enough for its bucket table, 16-byte
// aligned keys, H and output).
bool fused_ok(const dialsort_desc& d, const Cfg& c);

// Lay the batch out in a workspace whose aligned base is `base` (null: sizes
// only): [Ctl][arrays][states][units][per-array regions]; P.bytes is the
// workspace size needed (including alignment slack).
void plan_batch(const dialsort_desc* d, uint32_t count, const Cfg& cfg, char* base, Planned& P);

// The tables (arrays, zeroed states, units) as one block of table_bytes(P)
// bytes, to be copied to base + P.off_arrays.
size_t table_bytes(const Planned& P);
void write_tables(const Planned& P, char* host);

// Fill a plan for a batch whose tables are (or will be) in ws.
dialsort_status make_plan(const Planned& P, uint32_t count, const Cfg& cfg, void* ws, size_t ws_bytes,
                          dialsort_batch_plan* plan);

// Enqueue the clearing launch and the fused launch of a plan on s.
dialsort_status launch_fused(const dialsort_batch_plan& p, hipStream_t s);

// The configuration used when the caller gives none.
Cfg default_cfg(const dialsort_desc* d, uint32_t count);

}  // namespace dsb
