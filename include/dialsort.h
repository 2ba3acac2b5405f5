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
 * paper's implementation does (Sec. 9.2, Table "tab:struct_cost"). */
dialsort_status dialsort_sort(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H,
                              uint32_t *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace for dialsort_sort_batched over these descriptors. */
size_t dialsort_batched_workspace_bytes(const dialsort_desc *descs, uint32_t count);

/* dialsort_sort on every descriptor (host array of count entries) as one
 * persistent device launch.  Each array's H and out equal what dialsort_sort
 * gives for it alone.  The first device-detected error of any array is reported
 * by dialsort_status_sync().  descs is read during the call only. */
dialsort_status dialsort_sort_batched(const dialsort_desc *descs, uint32_t count, void *ws,
                                      size_t ws_bytes, hipStream_t stream);

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
 * out of range).  Static storage. */
const char *dialsort_launch_name(uint32_t i);

/* Text for a status code (static storage). */
const char *dialsort_strerror(dialsort_status status);

/* The hipError_t of the most recent failed HIP call in this thread (0 if none). */
int dialsort_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DIALSORT_H */
