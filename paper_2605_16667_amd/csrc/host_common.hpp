// Host helpers shared by the translation units of libdialsort: error and
// launch bookkeeping, alignment arithmetic, and the single-array launch
// sequence that the batched entry points fall back to.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/dialsort.h"

namespace dsh {

constexpr size_t ALIGN = 256;
constexpr uint64_t U_MAX = 1ull << 32;
constexpr uint64_t N_MAX = 0xFFFFFFFFull;

// Last failing HIP call of this host thread (dialsort_last_hip_error).
extern thread_local int g_last_hip_error;

// Measurement hook (dialsort_set_launch_events): per host thread, an optional
// caller-owned event array; events[i] is recorded on the launch stream just
// before launch i of the current call, events[count] after its last launch.
struct LaunchLog {
  hipEvent_t* ev = nullptr;
  uint32_t cap = 0;
  uint32_t* count = nullptr;
  uint32_t n = 0;
  std::vector<const char*> names;  // kernel of launch i (the first max(cap, 64) launches)
};
extern thread_local LaunchLog g_log;

inline void log_launch(const char* name, hipStream_t s) {
  if (g_log.ev && g_log.n + 1 < g_log.cap) (void)hipEventRecord(g_log.ev[g_log.n], s);
  if (g_log.n < g_log.names.size()) g_log.names[g_log.n] = name;
  ++g_log.n;
}

// Opens a public call: resets the launch log; on close records the end event.
struct CallScope {
  hipStream_t s;
  explicit CallScope(hipStream_t st) : s(st) { g_log.n = 0; }
  ~CallScope() {
    if (g_log.ev && g_log.n < g_log.cap) (void)hipEventRecord(g_log.ev[g_log.n], s);
    if (g_log.count) *g_log.count = g_log.n;
  }
};

#define DS_LAUNCH(kernel, grid, block, stream, ...)                      \
  do {                                                                   \
    ::dsh::log_launch(#kernel, stream);                                  \
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);     \
    hipError_t e_ = hipGetLastError();                                   \
    if (e_ != hipSuccess) {                                              \
      ::dsh::g_last_hip_error = (int)e_;                                 \
      return DIALSORT_EHIP;                                              \
    }                                                                    \
  } while (0)

#define DS_TRY(x)                          \
  do {                                     \
    dialsort_status st_ = (x);             \
    if (st_ != DIALSORT_OK) return st_;    \
  } while (0)

#define DS_HIP(x)                          \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) {                \
      ::dsh::g_last_hip_error = (int)e_;   \
      return DIALSORT_EHIP;                \
    }                                      \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline uint64_t cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }
inline bool aligned4(const void* p) { return ((uintptr_t)p & 3) == 0; }
inline bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!abytes || !bbytes) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bbytes && y < x + abytes;
}
inline char* ws_base(void* ws) { return (char*)align_up((uintptr_t)ws, ALIGN); }

// Argument checks of one array (dialsort_sort's rules).
dialsort_status check_desc(const dialsort_desc& d);

// The single-array launch sequences of dialsort_sort, one array after the other
// on `s`, each in a sub-workspace of loop_workspace_bytes(); the device status of
// every array is folded into the status word of ws.
size_t loop_workspace_bytes(const dialsort_desc* d, uint32_t count);
dialsort_status loop_run(const dialsort_desc* d, uint32_t count, void* ws, size_t ws_bytes, hipStream_t s);
// Running count P[0 .. U] of H (query.hip); ws sized by dialsort_prefix_workspace_bytes(U).
dialsort_status launch_prefix(const uint32_t* H, uint64_t U, uint64_t* P, void* ws, hipStream_t stream);

}  // namespace dsh
