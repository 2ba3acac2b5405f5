// libdialsort serving engine: sort requests of mixed n and U arrive over time
// and are run by continuous batching on device-resident buffers.
//
//   * Memory: the caller gives one device arena.  A request is admitted (FIFO)
//     when its footprint -- H (U counters) and its output (n keys) -- fits in
//     the arena; both stay resident until the caller releases the request.
//   * Batching: every poll retires the batches that finished, admits what
//     fits, and launches the admitted requests as one fused batched launch
//     (csrc/batch.hpp) on a free stream slot -- a lone request takes
//     dialsort_sort's own launch sequence instead; up to max_inflight batches run on
//     the device at once, on separate streams, so requests that arrive while
//     others are on the GPU start as soon as a slot and memory are free and
//     their work overlaps with the running batches.  A batch's workspace is
//     taken from the arena at launch and returned when it finishes.
//   * Launches never wait on the host: plan tables go to the device from pinned
//     staging with an asynchronous copy, the batch's device status comes back
//     the same way, and completion is read from an event.  Times are taken from
//     events against a start event, so a request's completion time is when its
//     batch finished on the device.
// Each request's H and output are exactly what dialsort_sort gives for it
// alone: the batch shares no counters between requests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/dialsort.h"
#include "batch_host.hpp"
#include "host_common.hpp"

using namespace dsh;
using namespace dsb;

namespace {

constexpr uint32_t MAX_SLOTS = 8;

// First-fit allocator of arena offsets (ALIGN-aligned), with coalescing.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes >= ALIGN) free_[0] = bytes / ALIGN * ALIGN;
    capacity_ = bytes / ALIGN * ALIGN;
  }
  bool alloc(size_t bytes, size_t* off) {
    const size_t need = std::max<size_t>(align_up(bytes, ALIGN), ALIGN);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        *off = it->first;
        const size_t rest = it->second - need;
        const size_t roff = it->first + need;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used_[*off] = need;
        return true;
      }
    }
    return false;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t capacity() const { return capacity_; }

 private:
  std::map<size_t, size_t> free_;
  std::unordered_map<size_t, size_t> used_;
  size_t capacity_ = 0;
};

enum ReqState : uint32_t { RQ_QUEUED = 0, RQ_ADMITTED = 1, RQ_RUNNING = 2, RQ_DONE = 3 };

struct Request {
  const uint32_t* keys;
  uint64_t n, U;
  size_t h_off = 0, o_off = 0;
  uint32_t state = RQ_QUEUED;
  dialsort_status status = DIALSORT_OK;
  double submit_ms = 0, launch_ms = 0, done_ms = 0, seen_ms = 0;
};

struct Slot {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> reqs;
  size_t ws_off = 0;
  char* pinned = nullptr;  // tables, then the batch's states as returned by the device
  size_t pinned_cap = 0;
  ds::BState* states = nullptr;
};

size_t footprint(uint64_t n, uint64_t U) { return align_up(U * 4, ALIGN) + align_up(std::max<uint64_t>(n, 1) * 4, ALIGN); }

}  // namespace

struct dialsort_server {
  std::mutex mu;
  int device = 0;
  char* arena = nullptr;
  Arena alloc;
  Cfg cfg;
  uint32_t max_batch = 256;
  std::vector<Slot> slots;
  hipEvent_t t0 = nullptr;
  std::chrono::steady_clock::time_point h0;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> queue;   // submitted, not admitted (FIFO)
  std::deque<uint64_t> ready;   // admitted, not launched (FIFO)
  uint32_t not_done = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - h0).count();
  }
};

namespace {

dialsort_status retire(dialsort_server* S) {
  const double seen = S->now_ms();
  for (Slot& sl : S->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    dialsort_status st = DIALSORT_OK;
    float ms = 0.f;
    if (q != hipSuccess || hipEventElapsedTime(&ms, S->t0, sl.done) != hipSuccess) {
      g_last_hip_error = (int)q;
      st = DIALSORT_EHIP;
      ms = (float)S->now_ms();
    }
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
      Request& r = S->reqs[sl.reqs[i]];
      dialsort_status rs = st;
      if (rs == DIALSORT_OK) {
        const uint32_t dev = ((volatile ds::BState*)sl.states)[i].status;
        if (dev & ds::ST_RANGE) rs = DIALSORT_ERANGE;
        else if (dev) rs = DIALSORT_EHIP;
      }
      r.state = RQ_DONE;
      r.status = rs;
      r.done_ms = ms;
      r.seen_ms = seen;
      --S->not_done;
    }
    sl.reqs.clear();
    S->alloc.release(sl.ws_off);
    sl.busy = false;
  }
  return DIALSORT_OK;
}

void admit(dialsort_server* S) {
  while (!S->queue.empty()) {
    Request& r = S->reqs[S->queue.front()];
    size_t h = 0, o = 0;
    if (!S->alloc.alloc(r.U * 4, &h)) break;
    if (!S->alloc.alloc(std::max<uint64_t>(r.n, 1) * 4, &o)) {
      S->alloc.release(h);
      break;
    }
    r.h_off = h;
    r.o_off = o;
    r.state = RQ_ADMITTED;
    S->ready.push_back(S->queue.front());
    S->queue.pop_front();
  }
}

// Pinned staging of a slot: at least `need` bytes (grown only while the slot
// is idle).
dialsort_status ensure_pinned(Slot& sl, size_t need) {
  if (sl.pinned_cap >= need) return DIALSORT_OK;
  if (sl.pinned) (void)hipHostFree(sl.pinned);
  sl.pinned = nullptr;
  sl.pinned_cap = 0;
  const size_t cap = std::max<size_t>(align_up(need, 1 << 20), 4 << 20);
  DS_HIP(hipHostMalloc((void**)&sl.pinned, cap, hipHostMallocDefault));
  sl.pinned_cap = cap;
  return DIALSORT_OK;
}

void mark_running(dialsort_server* S, Slot& sl, size_t k, size_t ws_off) {
  const double t = S->now_ms();
  sl.reqs.assign(S->ready.begin(), S->ready.begin() + k);
  for (uint64_t id : sl.reqs) {
    Request& r = S->reqs[id];
    r.state = RQ_RUNNING;
    r.launch_ms = t;
  }
  S->ready.erase(S->ready.begin(), S->ready.begin() + k);
  sl.ws_off = ws_off;
  sl.busy = true;
}

// A lone request runs dialsort_sort's own launch sequence: nothing to batch
// with, and no batch bookkeeping to pay for.
dialsort_status launch_single(dialsort_server* S, Slot& sl, bool* launched) {
  *launched = false;
  const Request& r = S->reqs[S->ready.front()];
  const size_t wsb = dialsort_workspace_bytes(r.n, r.U, DIALSORT_MODE_SORT);
  size_t ws_off = 0;
  if (!S->alloc.alloc(wsb, &ws_off)) return DIALSORT_OK;  // wait for memory
  dialsort_status st = ensure_pinned(sl, sizeof(ds::BState));
  if (st != DIALSORT_OK) {
    S->alloc.release(ws_off);
    return st;
  }
  sl.states = (ds::BState*)sl.pinned;
  char* ws = S->arena + ws_off;
  st = dialsort_sort(r.keys, r.n, r.U, (uint32_t*)(S->arena + r.h_off), (uint32_t*)(S->arena + r.o_off), ws, wsb,
                     sl.stream);
  hipError_t e = hipSuccess;
  if (st == DIALSORT_OK)
    e = hipMemcpyAsync(&sl.states[0].status, ws_base(ws) + offsetof(ds::Ctl, status), 4, hipMemcpyDeviceToHost,
                       sl.stream);
  if (st == DIALSORT_OK && e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    st = DIALSORT_EHIP;
  }
  if (st != DIALSORT_OK) {
    (void)hipStreamSynchronize(sl.stream);
    S->alloc.release(ws_off);
    return st;
  }
  mark_running(S, sl, 1, ws_off);
  *launched = true;
  return DIALSORT_OK;
}

dialsort_status launch_one(dialsort_server* S, Slot& sl, bool* launched) {
  *launched = false;
  if (S->ready.size() == 1) {
    DS_TRY(launch_single(S, sl, launched));
    if (*launched) return DIALSORT_OK;
    // no room for dialsort_sort's workspace: the fused form needs far less
  }
  size_t k = std::min<size_t>(S->ready.size(), S->max_batch);
  std::vector<dialsort_desc> d;
  Planned P;
  size_t ws_off = 0;
  for (;;) {
    d.resize(k);
    for (size_t i = 0; i < k; ++i) {
      const Request& r = S->reqs[S->ready[i]];
      d[i].keys = r.keys;
      d[i].n = r.n;
      d[i].U = r.U;
      d[i].H = (uint32_t*)(S->arena + r.h_off);
      d[i].out = (uint32_t*)(S->arena + r.o_off);
    }
    plan_batch(d.data(), (uint32_t)k, S->cfg, nullptr, P);
    if (S->alloc.alloc(P.bytes, &ws_off)) break;
    if (k == 1) return DIALSORT_OK;  // wait for memory
    k = (k + 1) / 2;
  }
  char* ws = S->arena + ws_off;
  char* base = ws_base(ws);
  plan_batch(d.data(), (uint32_t)k, S->cfg, base, P);
  const size_t tb = table_bytes(P);
  {
    const dialsort_status pst = ensure_pinned(sl, align_up(tb, 64) + k * sizeof(ds::BState));
    if (pst != DIALSORT_OK) {
      S->alloc.release(ws_off);
      return pst;
    }
  }
  write_tables(P, sl.pinned);
  sl.states = (ds::BState*)(sl.pinned + align_up(tb, 64));
  dialsort_batch_plan plan;
  dialsort_status st = make_plan(P, (uint32_t)k, S->cfg, ws, P.bytes, &plan);
  hipError_t e = hipSuccess;
  if (st == DIALSORT_OK) e = hipMemcpyAsync(base + P.off_arrays, sl.pinned, tb, hipMemcpyHostToDevice, sl.stream);
  if (st == DIALSORT_OK && e == hipSuccess) st = launch_fused(plan, sl.stream);
  if (st == DIALSORT_OK && e == hipSuccess)
    e = hipMemcpyAsync(sl.states, base + P.off_states, k * sizeof(ds::BState), hipMemcpyDeviceToHost, sl.stream);
  if (st == DIALSORT_OK && e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    st = DIALSORT_EHIP;
  }
  if (st != DIALSORT_OK) {
    // nothing of this batch is known to be enqueued correctly: wait for the
    // stream before the workspace goes back to the arena
    (void)hipStreamSynchronize(sl.stream);
    S->alloc.release(ws_off);
    return st;
  }
  mark_running(S, sl, k, ws_off);
  *launched = true;
  return DIALSORT_OK;
}

// Launch policy: while the admitted requests are no more than the free slots,
// each runs alone on its own slot (their launches overlap on the device); when
// more have piled up, the free slot takes all of them (up to max_batch) as one
// fused launch, which amortises per-request launch costs under load.
dialsort_status step(dialsort_server* S, bool* progress) {
  DS_TRY(retire(S));
  admit(S);
  *progress = false;
  for (Slot& sl : S->slots) {
    if (S->ready.empty()) break;
    if (sl.busy) continue;
    uint32_t free_slots = 0;
    for (const Slot& o : S->slots) free_slots += o.busy ? 0u : 1u;
    bool launched = false;
    if (S->ready.size() <= free_slots) {
      DS_TRY(launch_single(S, sl, &launched));
      if (!launched) DS_TRY(launch_one(S, sl, &launched));
    } else {
      DS_TRY(launch_one(S, sl, &launched));
    }
    if (!launched) break;
    *progress = true;
  }
  return DIALSORT_OK;
}

uint32_t busy_slots(const dialsort_server* S) {
  uint32_t b = 0;
  for (const Slot& sl : S->slots) b += sl.busy ? 1u : 0u;
  return b;
}

}  // namespace

extern "C" {

size_t dialsort_server_footprint(uint64_t n, uint64_t U) { return footprint(n, U); }

double dialsort_server_now_ms(const dialsort_server* S) { return S ? S->now_ms() : -1.0; }

dialsort_status dialsort_server_create(void* arena, size_t arena_bytes, const dialsort_server_config* config,
                                       dialsort_server** server) {
  if (!server || !arena || !config) return DIALSORT_EINVAL;
  if (!cfg_valid(config->batch) || config->max_inflight < 1 || config->max_inflight > MAX_SLOTS ||
      config->max_batch < 1)
    return DIALSORT_EINVAL;
  dialsort_server* S = new dialsort_server();
  S->cfg = to_cfg(config->batch);
  S->cfg.classes = false;  // a request completes with its whole launch
  S->max_batch = config->max_batch;
  S->arena = ws_base(arena);
  const size_t lost = (size_t)(S->arena - (char*)arena);
  S->alloc.reset(arena_bytes > lost ? arena_bytes - lost : 0);
  hipError_t e = hipGetDevice(&S->device);
  S->slots.resize(config->max_inflight);
  for (Slot& sl : S->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sl.done);
    // pinned staging now: a first allocation inside a launch would stall the
    // requests queued behind it
    if (e == hipSuccess && ensure_pinned(sl, 1) != DIALSORT_OK) e = hipErrorOutOfMemory;
  }
  if (e == hipSuccess) e = hipEventCreate(&S->t0);
  if (e == hipSuccess) e = hipEventRecord(S->t0, S->slots[0].stream);
  if (e == hipSuccess) e = hipEventSynchronize(S->t0);
  if (e != hipSuccess) {
    g_last_hip_error = (int)e;
    dialsort_server_destroy(S);
    return DIALSORT_EHIP;
  }
  S->h0 = std::chrono::steady_clock::now();
  *server = S;
  return DIALSORT_OK;
}

dialsort_status dialsort_server_destroy(dialsort_server* S) {
  if (!S) return DIALSORT_EINVAL;
  (void)hipSetDevice(S->device);
  for (Slot& sl : S->slots) {
    if (sl.busy && sl.done) (void)hipEventSynchronize(sl.done);
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  if (S->t0) (void)hipEventDestroy(S->t0);
  delete S;
  return DIALSORT_OK;
}

dialsort_status dialsort_server_submit(dialsort_server* S, const uint32_t* keys, uint64_t n, uint64_t U,
                                       uint64_t* id) {
  if (!S || !id) return DIALSORT_EINVAL;
  if (U == 0 || U > U_MAX || (n && !keys) || (n && !aligned16(keys))) return DIALSORT_EINVAL;
  if (n > N_MAX) return DIALSORT_EOVERFLOW;
  // H and the output will sit in the arena (aligned): only the keys and U
  // decide whether the fused launch takes the request
  dialsort_desc probe;
  probe.keys = keys;
  probe.n = n;
  probe.U = U;
  probe.H = (uint32_t*)(uintptr_t)ALIGN;
  probe.out = probe.H;
  if (!fused_ok(probe, S->cfg)) return DIALSORT_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  // a request that could never be admitted, even alone
  Planned P;
  plan_batch(&probe, 1, S->cfg, nullptr, P);
  // the fused form's workspace: a lone request falls back to it when
  // dialsort_sort's larger one does not fit
  if (footprint(n, U) + P.bytes + 2 * ALIGN > S->alloc.capacity()) return DIALSORT_EWORKSPACE;
  Request r;
  r.keys = keys;
  r.n = n;
  r.U = U;
  r.submit_ms = S->now_ms();
  const uint64_t rid = S->next_id++;
  S->reqs.emplace(rid, r);
  S->queue.push_back(rid);
  ++S->not_done;
  *id = rid;
  return DIALSORT_OK;
}

dialsort_status dialsort_server_poll(dialsort_server* S, uint32_t* pending) {
  if (!S) return DIALSORT_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  DS_HIP(hipSetDevice(S->device));
  bool progress = false;
  DS_TRY(step(S, &progress));
  if (pending) *pending = S->not_done;
  return DIALSORT_OK;
}

dialsort_status dialsort_server_drain(dialsort_server* S) {
  if (!S) return DIALSORT_EINVAL;
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      DS_HIP(hipSetDevice(S->device));
      bool progress = false;
      DS_TRY(step(S, &progress));
      if (S->not_done == 0) return DIALSORT_OK;
      // nothing running and nothing could start: the arena is held by
      // released-late results
      if (busy_slots(S) == 0 && !progress) return DIALSORT_EWORKSPACE;
      // block on the earliest busy slot instead of spinning
      for (Slot& sl : S->slots)
        if (sl.busy) {
          DS_HIP(hipEventSynchronize(sl.done));
          break;
        }
    }
  }
}

dialsort_status dialsort_server_info(dialsort_server* S, uint64_t id, dialsort_request_info* info) {
  if (!S || !info) return DIALSORT_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return DIALSORT_EINVAL;
  const Request& r = it->second;
  std::memset(info, 0, sizeof(*info));
  info->state = r.state;
  info->status = r.status;
  info->n = r.n;
  info->U = r.U;
  if (r.state >= RQ_ADMITTED) {
    info->H = (uint32_t*)(S->arena + r.h_off);
    info->out = (uint32_t*)(S->arena + r.o_off);
  }
  info->submit_ms = r.submit_ms;
  info->launch_ms = r.launch_ms;
  info->done_ms = r.done_ms;
  info->seen_ms = r.seen_ms;
  return DIALSORT_OK;
}

dialsort_status dialsort_server_release(dialsort_server* S, uint64_t id) {
  if (!S) return DIALSORT_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end() || it->second.state != RQ_DONE) return DIALSORT_EINVAL;
  S->alloc.release(it->second.h_off);
  S->alloc.release(it->second.o_off);
  S->reqs.erase(it);
  return DIALSORT_OK;
}

}  // extern "C"
