/*
 * dialsort.h -- C ABI of libdialsort.so, the MI355X (gfx950) DialSort hot path.
 *
 * DialSort (Narvaez, 2026) sorts n integer keys drawn from a bounded universe
 * [0, U) by using every key as its own address: ingestion counts the keys into a
 * histogram H[0, U) (Sec. 3.3, Eq. (1)), and H -- not the output array -- is the
 * canonical ordered state (Sec. 3.3, "Canonical ordered state").  The optional
 * ordered projection expands H into the sorted array, emitting k exactly H[k]
 * times for k = 0 .. U-1 (Sec. 3.3, Eq. (2)).  Concurrent updates of one key are
 * merged additively using equality tests only, the on-chip analogue of the
 * Conflict Resolution Network (Sec. 6, Eqs. (3)/(4), Lemma "lem:crn").
 *
 * Conventions shared by every entry point
 *   - Keys, H and outputs are uint32.  All array pointers are DEVICE pointers
 *     owned by the caller; the library never allocates, frees or retains them.
 *     Every uint32 pointer must be 4-byte aligned (EINVAL otherwise); 16-byte
 *     alignment is faster but not required.
 *   - ws / ws_bytes: a caller-owned device workspace of at least the size that
 *     the matching *_workspace_bytes query returns.  One workspace serves one call
 *     at a time; calls that share a workspace must be stream-ordered.  Calls with
 *     distinct workspaces are thread-safe.
 *   - stream: every call only enqueues work on `stream` (0 = the null stream) and
 *     returns; nothing is synchronised.  Argument errors are detected on the host
 *     and returned at once, before anything is enqueued.  Errors that depend on
 *     key values (ERANGE) or on H (EOVERFLOW in dialsort_reconstruct) are
 *     detected on the device and read back with dialsort_status_sync().
 *   - U may be any value in [1, 2^32]; powers of two are not required.
 *   - After a device-detected error the contents of H and of the output are
 *     unspecified.
 */
#ifndef DIALSORT_H
#define DIALSORT_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DIALSORT_OK = 0,
    DIALSORT_EINVAL = 1,     /* null pointer with nonzero size, U == 0 or U > 2^32,
                                misaligned pointer, or out partially overlapping keys */
    DIALSORT_ERANGE = 2,     /* some key >= U: the method is defined only on [0, U)
                                (Sec. 16, "Bounded universe required") */
    DIALSORT_EOVERFLOW = 3,  /* n > 2^32 - 1 (counts are uint32), or sum(H) > out_cap */
    DIALSORT_EWORKSPACE = 4, /* ws is null or ws_bytes is below the required size */
    DIALSORT_EHIP = 5        /* a HIP runtime call failed; see dialsort_last_hip_error() */
} dialsort_status;

/* Modes for the workspace query. */
#define DIALSORT_MODE_HISTOGRAM 0  /* dialsort_histogram */
#define DIALSORT_MODE_SORT 1       /* dialsort_sort */
#define DIALSORT_MODE_RECONSTRUCT 2 /* dialsort_reconstruct: pass n = out_cap */
#define DIALSORT_MODE_ACCUMULATE 3  /* dialsort_histogram_accumulate */

/* One array of a batch: the same meaning as the arguments of dialsort_sort.
 * out may equal keys (in place); any other overlap is EINVAL. */
typedef struct dialsort_desc {
    const uint32_t *keys; /* n keys in [0, U) */
    uint64_t n;
    uint64_t U;
    uint32_t *H;   /* U counters, fully overwritten */
    uint32_t *out; /* n sorted keys */
} dialsort_desc;

/* Bytes of device workspace needed by one call with these sizes. */
size_t dialsort_workspace_bytes(uint64_t n, uint64_t U, int mode);

/* Ingestion only (Sec. 3.3, Eq. (1)): H[k] := |{ i : keys[i] == k }| for every
 * k in [0, U).  H is overwritten, not accumulated; the caller need not clear
 * it.  n == 0 gives H == 0.  n > 2^32 - 1 is EOVERFLOW. */
dialsort_status dialsort_histogram(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H,
                                   void *ws, size_t ws_bytes, hipStream_t stream);

/* Keys from a universe that starts at lo: the order-isomorphism phi(x) =
 * x - lo (mod 2^32) of the General Self-Indexing Principle (Sec. 3.4,
 * Proposition "General Self-Indexing Principle") maps [lo, lo + U) onto
 * [0, U) in order, and its inverse lo + k is applied as the projection writes.
 * H[k] counts the key lo + k; out receives the keys themselves in phi order.
 * lo = 0 is dialsort_histogram / dialsort_sort.  Signed int32 keys are the
 * case lo = 0x80000000 (phi flips the sign bit) with U = 2^32, or lo = the
 * smallest value's bit pattern for a narrower signed range.  A key outside
 * [lo, lo + U) (mod 2^32) is ERANGE.  Workspace sizes and every other
 * convention are those of dialsort_histogram / dialsort_sort. */
dialsort_status dialsort_histogram_offset(const uint32_t *keys, uint64_t n, uint32_t lo, uint64_t U, uint32_t *H,
                                          void *ws, size_t ws_bytes, hipStream_t stream);
dialsort_status dialsort_sort_offset(const uint32_t *keys, uint64_t n, uint32_t lo, uint64_t U, uint32_t *H,
                                     uint32_t *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Keys given as indices phi(s) in [0, U) of a finite totally ordered domain,
 * with phi^-1 as a table (Sec. 3.4, the General Self-Indexing Principle: the
 * projection emits phi^-1(k) H[k] times, and outside the integers a lookup
 * table serves as phi^-1).  lut holds U 32-bit values, lut[k] = phi^-1(k)
 * (device memory, read only).  H is the histogram of the indices, as in
 * dialsort_sort, and out[0 .. n) receives lut[k] for the indices in
 * nondecreasing order: the elements in the domain's order when lut is
 * increasing.  lut must not overlap H or out; out may equal keys.  An index
 * >= U is ERANGE.  Workspace: dialsort_workspace_bytes(n, U,
 * DIALSORT_MODE_SORT). */
dialsort_status dialsort_sort_lut(const uint32_t *keys, uint64_t n, uint64_t U, const uint32_t *lut, uint32_t *H,
                                  uint32_t *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* The smallest and the largest key, compared as int32 when is_signed, else as
 * uint32: minmax[0] = min, minmax[1] = max (two 32-bit words of device
 * memory, written on `stream`).  They give the smallest offset map of Sec. 3.4
 * that holds the keys (the min-max choice of phi): lo = min, U = max - min + 1
 * (as a 64-bit count) for dialsort_sort_offset.  n == 0 leaves min above max:
 * the pair (0xFFFFFFFF, 0), or (0x7FFFFFFF, 0x80000000) when is_signed.  No
 * workspace; minmax must not overlap keys. */
dialsort_status dialsort_key_range(const uint32_t *keys, uint64_t n, int is_signed, uint32_t *minmax,
                                   hipStream_t stream);

/* Accumulating ingestion, for keys that arrive in pieces (streaming): H[k] +=
 * |{ i : keys[i] == k }| for every k in [0, U), so that ingesting a key stream
 * piece by piece leaves in H the histogram of the whole stream (Eq. (1) is a
 * sum over the keys, and the CRN merge is additive: Sec. 6, Lemma "lem:crn").
 * The paper notes that streaming can overlap ingestion and projection given
 * extra synchronisation (Sec. 4, remark after the complexity theorem); here
 * pieces are ordered on `stream`, and dialsort_reconstruct projects H once
 * the stream ends.  A bin that would pass 2^32 - 1 is reported as EOVERFLOW
 * by dialsort_status_sync() (H is then unspecified), and so is a key >= U as
 * ERANGE.  The workspace size is dialsort_workspace_bytes(n, U,
 * DIALSORT_MODE_ACCUMULATE). */
dialsort_status dialsort_histogram_accumulate(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H,
                                              void *ws, size_t ws_bytes, hipStream_t stream);

/* A stream of keys sorted in tumbling windows, with ingestion and projection
 * overlapped (the streaming remark after the complexity theorem of Sec. 4):
 * window w is keys[w*window_n .. (w+1)*window_n), w < count; its histogram
 * (Eq. (1)) goes to H + (w mod 2)*U and its ordered projection (Eq. (2)) to
 * out + w*window_n.  Ingestions run in order on `ingest` and projections on
 * `project`: window w + 1 is ingested while window w is projected, and a
 * histogram is reused only after its previous window's projection.  H holds
 * 2U counters; on completion it holds the histograms of the last two windows.
 * keys, out and H must not overlap (out == keys is EINVAL here).  Passing the
 * same stream twice gives the serial order.  The first ingestion waits for
 * the work already on `project` (so a previous call's projections, which read
 * the same H and workspace, finish first); work already on `ingest` is not
 * ordered against `project`: order it with an event if it produces the keys.
 * Completion of everything is ordered before later work on `project`.  The workspace (dialsort_windows_workspace_bytes) holds the
 * combined device status read by dialsort_status_sync(ws, project): a key >= U
 * in any window is ERANGE. */
size_t dialsort_windows_workspace_bytes(uint64_t window_n, uint64_t U);
dialsort_status dialsort_sort_windows(const uint32_t *keys, uint64_t window_n, uint32_t count, uint64_t U,
                                      uint32_t *H, uint32_t *out, void *ws, size_t ws_bytes, hipStream_t ingest,
                                      hipStream_t project);

/* Ordered projection only (Sec. 3.3, Eq. (2)): writes k exactly H[k] times for
 * k = 0 .. U-1 into out, in ascending k, stopping after out_cap elements.  The
 * number of elements is min(sum H, out_cap); sum H > out_cap is reported as
 * EOVERFLOW by dialsort_status_sync() (the first out_cap elements are still
 * written).  Read sum H with dialsort_result_total().  out_cap must be below
 * 2^62.  The workspace size is dialsort_workspace_bytes(out_cap, U,
 * DIALSORT_MODE_RECONSTRUCT). */
dialsort_status dialsort_reconstruct(const uint32_t *H, uint64_t U, uint32_t *out, uint64_t out_cap,
                                     void *ws, size_t ws_bytes, hipStream_t stream);

/* Ingestion followed by the ordered projection: H as in dialsort_histogram and
 * out[0 .. n) = the keys in nondecreasing order (Theorem "thm:correct").  out may
 * equal keys: the projection is then written in place over the input, as the
 * paper's implementation does (Sec. 9.2, Table "tab:struct_cost").  A small sort
 * with U <= 65536 (up to 16 keys per 1024 bins, at most 2^24 keys) is one kernel
 * launch whose scan blocks wait for flags carrying a value the host draws per
 * call; on a stream that is capturing a graph (where replays would repeat that
 * value) the same sort is enqueued as two launches instead, so a captured sort
 * replays exactly. */
dialsort_status dialsort_sort(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H,
                              uint32_t *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---- Batches of independent arrays ------------------------------------------
 *
 * A batch is a host array of `count` descriptors, each an independent
 * dialsort_sort problem with its own n, U, H and output.  Every array's H and
 * output equal what dialsort_sort gives for it alone (the batch shares no
 * counters between arrays).  The first device-detected error of any array is
 * reported by dialsort_status_sync() on the batch workspace, after which the
 * contents of every H and output of the batch are unspecified.  Batching is not
 * part of the paper, which sorts one array; it applies the method of Sec. 3.3
 * to many arrays at once.
 *
 * The fused form runs the whole batch as ONE persistent kernel launch (plus a
 * small launch that clears its counters) over a table of work units: every
 * array's ingestion (Eq. (1)), then its counting and scan, then its projection
 * (Eq. (2)), with per-array completion counters ordering the phases.  It takes
 * arrays with U <= 1024 * 2^log2_width whose keys, H and output are 16-byte
 * aligned; dialsort_batch_prepare() rejects any other array with EINVAL, and
 * dialsort_sort_batched() then falls back to the per-array launch sequences of
 * dialsort_sort_each(). */

/* Tuning parameters of the fused launch. */
typedef struct dialsort_batch_config {
    uint32_t block;       /* threads per workgroup: 512 or 1024 */
    uint32_t log2_width;  /* U-partition width W = 2^log2_width bins, 14..16: an
                             array with U <= W is counted in LDS sub-histograms,
                             a larger one through the U-range-partitioned path
                             with buckets of W bins */
    uint64_t chunk_keys;  /* keys per private LDS sub-histogram, a power of two
                             in [2^16, 2^22]: an array with U <= W gets
                             ceil(n / chunk_keys) private copies (privatization
                             depth), summed before its scan */
} dialsort_batch_config;

/* A prepared batch: plain data, owned by the caller, filled by
 * dialsort_batch_prepare().  It refers to the workspace and to the device
 * buffers named by the descriptors, which must stay allocated while the plan
 * is launched. */
typedef struct dialsort_batch_plan {
    dialsort_batch_config config;
    uint32_t count;         /* arrays */
    uint32_t units;         /* work units of one launch */
    uint32_t grid;          /* persistent workgroups of the fused kernel */
    uint32_t fill_units;    /* the last fill_units of the units: fill units of
                               the late size classes, run by a second kernel
                               of small workgroups right after the fused one */
    uint64_t units_offset;  /* where the unit table sits in the workspace */
    void *ws;
    size_t ws_bytes;
} dialsort_batch_plan;

/* Workspace for any of the batched calls over these descriptors (every
 * configuration and the per-array form); 0 if some U is 0 or above 2^32. */
size_t dialsort_batched_workspace_bytes(const dialsort_desc *descs, uint32_t count);

/* Plans the fused launch of a batch with `config` (NULL: the configuration
 * that dialsort_batch_autotune() found for a batch of these sizes on this
 * device, else the built-in default) and copies its tables into ws.  This call
 * synchronises `stream` (the tables are uploaded from host memory).  descs is
 * read during the call only.  Errors: EINVAL (bad descriptor, array outside
 * the fused form, bad config), EWORKSPACE, EHIP. */
dialsort_status dialsort_batch_prepare(const dialsort_desc *descs, uint32_t count,
                                       const dialsort_batch_config *config, void *ws,
                                       size_t ws_bytes, hipStream_t stream,
                                       dialsort_batch_plan *plan);

/* Enqueues the prepared batch on `stream`: three kernel launches at most
 * (clear, fused, late fills), no host
 * synchronisation, no allocation and no copy, so the call may be captured into
 * a HIP graph (hipStreamBeginCapture) and replayed; each launch recomputes
 * every H and output from the keys.  One plan (one workspace) must not be
 * launched twice concurrently. */
dialsort_status dialsort_batch_launch(const dialsort_batch_plan *plan, hipStream_t stream);

/* Prepare + launch in one call (synchronises `stream` for the table upload),
 * falling back to dialsort_sort_each() when some array is outside the fused
 * form. */
dialsort_status dialsort_sort_batched(const dialsort_desc *descs, uint32_t count, void *ws,
                                      size_t ws_bytes, hipStream_t stream);

/* The plain form: dialsort_sort's own launch sequence for every array in turn,
 * stream-ordered, in one shared sub-workspace (about four launches per array). */
dialsort_status dialsort_sort_each(const dialsort_desc *descs, uint32_t count, void *ws,
                                   size_t ws_bytes, hipStream_t stream);

/* Times every candidate configuration (block 512/1024 x log2_width 14/15/16 x
 * chunk_keys 2^18/2^20/2^22, those that take every array) on this batch --
 * each candidate runs the whole batch three times, so every H and output is
 * written -- stores the fastest in *best and remembers it for batches of the
 * same sizes on this device (the library's only tuning state; besides it the
 * library keeps the one-launch sort's epoch sequence, see dialsort_sort).
 * Synchronises
 * `stream`.  ws as for dialsort_batched_workspace_bytes(). */
dialsort_status dialsort_batch_autotune(const dialsort_desc *descs, uint32_t count, void *ws,
                                        size_t ws_bytes, hipStream_t stream,
                                        dialsort_batch_config *best);

/* The configuration dialsort_batch_prepare() would use for config == NULL. */
dialsort_status dialsort_batch_default_config(const dialsort_desc *descs, uint32_t count,
                                              dialsort_batch_config *config);

/* After a launch of `plan` has been enqueued: waits for `stream` and stores,
 * for the first `count` arrays, the time in ms from the start of the launch's
 * first work unit to the end of the array's last one (array_ms[i]), in
 * *launch_ms (if not NULL) the time to the end of the last unit of the whole
 * launch, and in unit_ms[0..11] (if not NULL), for the unit types ingestion
 * (LDS), ingestion (partition), row sum + scan, bucket, fill in the fused
 * kernel, fill in the late-fill kernel, the workgroup-milliseconds spent
 * working (unit_ms[2t]) and waiting for other units (unit_ms[2t+1], always 0
 * for the late fills, which never wait).  Read from the device wall clock. */
dialsort_status dialsort_batch_times(const dialsort_batch_plan *plan, hipStream_t stream,
                                     double *array_ms, uint32_t count, double *launch_ms,
                                     double *unit_ms);

/* ---- Serving: continuous batching of sort requests ----------------------------
 *
 * A server runs sort requests of mixed n and U that arrive over time.  It owns
 * a device arena given by the caller and admits requests first-in first-out
 * by their HBM footprint: a request's H (U counters) and output (n keys) are
 * reserved in the arena at admission and stay resident there until the caller
 * releases the request, so later work can read the canonical histogram
 * (Sec. 3.3) without moving it.  Each poll retires finished batches, admits
 * what fits, and launches every admitted request (up to max_batch) as one
 * fused batched launch on a free stream; up to max_inflight batches run on the
 * device at once, on separate streams, so work that arrives while others run
 * overlaps with them.  A request's H and output equal dialsort_sort's for the
 * same keys, whatever else is in its batch.  Keys are read from the caller's
 * device buffer (16-byte aligned) and must stay unchanged until the request is
 * done.  A server is used from one host thread at a time (calls are
 * serialised by a lock).  Serving is not part of the paper; it runs the
 * method of Sec. 3.3 for many clients. */

typedef struct dialsort_server dialsort_server;

typedef struct dialsort_server_config {
    dialsort_batch_config batch;  /* configuration of every fused launch */
    uint32_t max_inflight;        /* batches on the device at once: 1..8 (one stream each) */
    uint32_t max_batch;           /* requests per batch, >= 1 */
} dialsort_server_config;

#define DIALSORT_REQ_QUEUED 0   /* waiting for arena space */
#define DIALSORT_REQ_ADMITTED 1 /* H and output reserved, not launched yet */
#define DIALSORT_REQ_RUNNING 2  /* in a batch on the device */
#define DIALSORT_REQ_DONE 3     /* H and output written (see status) */

typedef struct dialsort_request_info {
    uint32_t state;          /* DIALSORT_REQ_* */
    dialsort_status status;  /* once done: OK, or ERANGE if a key is >= U */
    uint32_t *H;             /* once admitted: the request's U counters in the arena */
    uint32_t *out;           /* once admitted: its n output keys in the arena */
    uint64_t n, U;
    double submit_ms;        /* times in ms since dialsort_server_create: submission, */
    double launch_ms;        /* launch of its batch (host clock) and end of its batch */
    double done_ms;          /* on the device (event clock) */
    double seen_ms;          /* host clock: when a poll or drain first found its batch
                                finished (the time a caller can observe completion;
                                comparable with submit_ms and dialsort_server_now_ms) */
} dialsort_request_info;

/* The server's host clock: ms since dialsort_server_create, the clock of
 * submit_ms, launch_ms and seen_ms.  Returns -1 for a null server. */
double dialsort_server_now_ms(const dialsort_server *server);

/* Arena bytes a request of this size holds from admission to release. */
size_t dialsort_server_footprint(uint64_t n, uint64_t U);

/* Creates a server on the current device.  arena: device memory owned by the
 * caller, kept allocated until dialsort_server_destroy returns.  Creates
 * max_inflight streams and events, and 4 MiB of pinned host staging per
 * stream (grown, while its stream is idle, when a batch's tables need more). */
dialsort_status dialsort_server_create(void *arena, size_t arena_bytes, const dialsort_server_config *config,
                                       dialsort_server **server);

/* Waits for every batch on the device, then frees the server. */
dialsort_status dialsort_server_destroy(dialsort_server *server);

/* Queues a request; nothing is enqueued on the device before the next poll.
 * EINVAL: bad arguments, or U above what the fused launch of the configuration
 * takes; EOVERFLOW: n > 2^32 - 1; EWORKSPACE: the request cannot fit in the
 * arena even alone. */
dialsort_status dialsort_server_submit(dialsort_server *server, const uint32_t *keys, uint64_t n, uint64_t U,
                                       uint64_t *id);

/* One non-blocking step: retire, admit, launch.  *pending (if not NULL)
 * receives the number of submitted requests not done yet. */
dialsort_status dialsort_server_poll(dialsort_server *server, uint32_t *pending);

/* Polls until every submitted request is done, waiting on the device in
 * between.  EWORKSPACE if nothing is running and nothing can start because the
 * arena is held by done requests that were not released. */
dialsort_status dialsort_server_drain(dialsort_server *server);

/* State, status, buffers and times of a request (EINVAL for an unknown or
 * released id). */
dialsort_status dialsort_server_info(dialsort_server *server, uint64_t id, dialsort_request_info *info);

/* Returns a done request's H and output to the arena (EINVAL if the request is
 * unknown or not done). */
dialsort_status dialsort_server_release(dialsort_server *server, uint64_t id);

/* Waits for `stream` and returns the device-detected status of the last call
 * that used ws (DIALSORT_OK, DIALSORT_ERANGE or DIALSORT_EOVERFLOW). */
dialsort_status dialsort_status_sync(const void *ws, hipStream_t stream);

/* Waits for `stream` and stores in *total the sum of H computed by the last
 * dialsort_reconstruct or dialsort_sort that used ws (saturated at 2^62 - 1). */
dialsort_status dialsort_result_total(const void *ws, hipStream_t stream, uint64_t *total);

/* Measurement hook, for benchmarks and profilers.  While set, every later call
 * on this host thread records events[i] on its stream just before its i-th
 * kernel launch (i < cap - 1) and one more event after its last launch, and
 * stores the call's number of launches in *count (if count is not null).  The
 * caller creates the events (hipEventCreate) and keeps them alive while the hook
 * is set; events == NULL switches the hook off.  cap < 2 with non-null events is
 * EINVAL.  The hook never changes what a call computes. */
dialsort_status dialsort_set_launch_events(hipEvent_t *events, uint32_t cap, uint32_t *count);

/* Kernel name of launch i of the last call on this host thread (NULL when i is
 * out of range or not below max(cap, 64) of the hook).  Static storage. */
const char *dialsort_launch_name(uint32_t i);

/* Text for a status code (static storage). */
const char *dialsort_strerror(dialsort_status status);

/* The hipError_t of the most recent failed HIP call in this thread (0 if none). */
int dialsort_last_hip_error(void);

/* ---- Queries on H ------------------------------------------------------------
 *
 * H is the canonical ordered state (Sec. 3.3, the paragraph on the canonical
 * ordered state): frequency(k), presence(k) and range-count(a, b) are answered
 * from H without building the ordered projection.  range-count and select read
 * the running count P[k] = H[0] + ... + H[k-1] (k = 0 .. U), built once by
 * dialsort_prefix; select(r) is the element at position r of the projection
 * (Eq. (2)) read without writing it.  H and P may have come from any source
 * (dialsort_histogram, a batch, a served request, the caller).  Every query
 * call enqueues one kernel on `stream` and returns; q, a, b, r and out are
 * device arrays of nq entries owned by the caller.  nq == 0 enqueues nothing. */

/* out[i] = H[q[i]] when q[i] < U, else 0 (a key outside the universe occurs 0
 * times).  H: U uint32; q, out: nq uint32, 4-byte aligned. */
dialsort_status dialsort_query_frequency(const uint32_t *H, uint64_t U, const uint32_t *q, uint64_t nq,
                                         uint32_t *out, hipStream_t stream);

/* out[i] = 1 when q[i] < U and H[q[i]] > 0, else 0 (the presence test of Sec.
 * 2.6, on the ingested state).  out: nq bytes. */
dialsort_status dialsort_query_presence(const uint32_t *H, uint64_t U, const uint32_t *q, uint64_t nq,
                                        uint8_t *out, hipStream_t stream);

/* Bytes of device workspace for dialsort_prefix (0 for U outside [1, 2^32]). */
size_t dialsort_prefix_workspace_bytes(uint64_t U);

/* P[k] = H[0] + ... + H[k-1] for k = 0 .. U: P has U + 1 uint64 entries,
 * 8-byte aligned, not overlapping H; P[U] = sum H.  Sums saturate at
 * 2^62 - 1 (never reached by a histogram of at most 2^32 - 1 keys).  One
 * workspace serves one call at a time. */
dialsort_status dialsort_prefix(const uint32_t *H, uint64_t U, uint64_t *P, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* out[i] = the number of keys in [a[i], b[i]) = P[min(b, U)] - P[min(a, b, U)]:
 * bounds past U are cut at U and a >= b counts nothing.  P from
 * dialsort_prefix; a, b, out: nq uint64, 8-byte aligned. */
dialsort_status dialsort_query_range_count(const uint64_t *P, uint64_t U, const uint64_t *a, const uint64_t *b,
                                           uint64_t nq, uint64_t *out, hipStream_t stream);

/* out[i] = the element at position r[i] of the ordered projection (Eq. (2)):
 * the k with P[k] <= r[i] < P[k + 1]; 0xFFFFFFFF when r[i] >= P[U].  P from
 * dialsort_prefix; r: nq uint64 (8-byte aligned), out: nq uint32. */
dialsort_status dialsort_query_select(const uint64_t *P, uint64_t U, const uint64_t *r, uint64_t nq,
                                      uint32_t *out, hipStream_t stream);

/* ---- DialSort-Radix: the whole 32-bit range ----------------------------------
 *
 * LSD, base 256, four passes, no order comparison (Sec. 8, "Full int32 range",
 * Table "tab:radix").  One read of the keys counts all four 8-bit digits
 * (Eq. (1) per digit); the running count of each digit histogram gives where
 * each digit starts (Eq. (2)); each pass then places every key stably at its
 * digit's start plus the count of that digit among the keys before it.
 * out[0 .. n) = the keys in ascending order: as uint32, or, with
 * is_signed != 0, as int32 (the sign bit is flipped on the first load and back
 * on the last store, the phi of Sec. 3.4).  No histogram over the 2^32 keys is
 * formed, so no key is out of range.  out may equal keys; any other overlap is
 * EINVAL.  n > 2^32 - 1 is EOVERFLOW.  The workspace (device memory, at least
 * dialsort_radix_workspace_bytes(n) bytes, contents not preserved) holds a
 * second copy of the keys and the per-tile digit counts. */
size_t dialsort_radix_workspace_bytes(uint64_t n);
dialsort_status dialsort_sort_radix(const uint32_t *keys, uint64_t n, int is_signed, uint32_t *out, void *ws,
                                    size_t ws_bytes, hipStream_t stream);

/* ---- Sorting without any allocation -----------------------------------------
 *
 * For callers that cannot allocate device memory or pass a workspace (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * dialsort_sort with the workspace taken from a 64 MiB array that the library
 * holds on each device from its load until the process ends.  Same arguments,
 * results and in-place rule as dialsort_sort, without ws; a sort whose
 * dialsort_workspace_bytes(n, U, DIALSORT_MODE_SORT) exceeds 64 MiB returns
 * EWORKSPACE before anything is enqueued.  status (device memory, 4-byte aligned,
 * may be null): receives the call's device status word once the sort has run
 * (0 = OK; bit 0 set = a key >= U, as ERANGE from dialsort_status_sync).
 * Nothing is allocated: no hipMalloc or hipFree, no allocating library routine.
 * Every call on a device shares that device's array and clears what must start
 * at zero; calls that overlap on one device (different streams, or threads
 * without ordering between their streams) race and give undefined results. */
dialsort_status dialsort_sort_noalloc(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H, uint32_t *out,
                                      uint32_t *status, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DIALSORT_H */
