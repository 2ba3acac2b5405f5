"""Python binding of libdialsort.so, the MI355X (gfx950) DialSort hot path.

The functions carry the names of the C ABI in include/dialsort.h and only
marshal arguments: torch tensors provide device memory and
``torch.cuda.current_stream()`` the stream; every step of the method runs in the
HIP kernels of the library.  There is no fallback: if the library is missing
the import of this binding fails.

Keys, H and outputs are 1-D ``torch.int32`` (or ``torch.uint32``) CUDA tensors
whose bits are uint32 values.  Each function returns the C status code
(``DIALSORT_OK`` == 0); ``check()`` turns a nonzero code into an exception.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

DIALSORT_OK, DIALSORT_EINVAL, DIALSORT_ERANGE, DIALSORT_EOVERFLOW, DIALSORT_EWORKSPACE, DIALSORT_EHIP = range(6)
DIALSORT_MODE_HISTOGRAM, DIALSORT_MODE_SORT, DIALSORT_MODE_RECONSTRUCT, DIALSORT_MODE_ACCUMULATE = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdialsort.so")


class DialSortError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"dialsort status {status}: {dialsort_strerror(status)}")
        self.status = status


class dialsort_desc(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("U", ctypes.c_uint64),
                ("H", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class dialsort_batch_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("log2_width", ctypes.c_uint32), ("chunk_keys", ctypes.c_uint64)]


class dialsort_batch_plan(ctypes.Structure):
    _fields_ = [("config", dialsort_batch_config), ("count", ctypes.c_uint32), ("units", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("fill_units", ctypes.c_uint32), ("units_offset", ctypes.c_uint64),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class dialsort_server_config(ctypes.Structure):
    _fields_ = [("batch", dialsort_batch_config), ("max_inflight", ctypes.c_uint32), ("max_batch", ctypes.c_uint32)]


class dialsort_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_uint32), ("status", ctypes.c_int), ("H", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("U", ctypes.c_uint64), ("submit_ms", ctypes.c_double),
                ("launch_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("seen_ms", ctypes.c_double)]


DIALSORT_REQ_QUEUED, DIALSORT_REQ_ADMITTED, DIALSORT_REQ_RUNNING, DIALSORT_REQ_DONE = range(4)


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python paper_2605_16667_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    u64, p, sz, st = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    sig = {
        "dialsort_workspace_bytes": (sz, [u64, u64, ctypes.c_int]),
        "dialsort_histogram": (st, [p, u64, u64, p, p, sz, p]),
        "dialsort_histogram_accumulate": (st, [p, u64, u64, p, p, sz, p]),
        "dialsort_histogram_offset": (st, [p, u64, ctypes.c_uint32, u64, p, p, sz, p]),
        "dialsort_sort_offset": (st, [p, u64, ctypes.c_uint32, u64, p, p, p, sz, p]),
        "dialsort_sort_lut": (st, [p, u64, u64, p, p, p, p, sz, p]),
        "dialsort_key_range": (st, [p, u64, ctypes.c_int, p, p]),
        "dialsort_windows_workspace_bytes": (sz, [u64, u64]),
        "dialsort_sort_windows": (st, [p, u64, ctypes.c_uint32, u64, p, p, p, sz, p, p]),
        "dialsort_reconstruct": (st, [p, u64, p, u64, p, sz, p]),
        "dialsort_sort": (st, [p, u64, u64, p, p, p, sz, p]),
        "dialsort_batched_workspace_bytes": (sz, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32]),
        "dialsort_sort_batched": (st, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32, p, sz, p]),
        "dialsort_sort_each": (st, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32, p, sz, p]),
        "dialsort_batch_prepare": (st, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32,
                                        ctypes.POINTER(dialsort_batch_config), p, sz, p,
                                        ctypes.POINTER(dialsort_batch_plan)]),
        "dialsort_batch_launch": (st, [ctypes.POINTER(dialsort_batch_plan), p]),
        "dialsort_batch_autotune": (st, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32, p, sz, p,
                                         ctypes.POINTER(dialsort_batch_config)]),
        "dialsort_batch_default_config": (st, [ctypes.POINTER(dialsort_desc), ctypes.c_uint32,
                                               ctypes.POINTER(dialsort_batch_config)]),
        "dialsort_batch_times": (st, [ctypes.POINTER(dialsort_batch_plan), p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
        "dialsort_server_footprint": (sz, [u64, u64]),
        "dialsort_server_now_ms": (ctypes.c_double, [p]),
        "dialsort_server_create": (st, [p, sz, ctypes.POINTER(dialsort_server_config), ctypes.POINTER(p)]),
        "dialsort_server_destroy": (st, [p]),
        "dialsort_server_submit": (st, [p, p, u64, u64, ctypes.POINTER(u64)]),
        "dialsort_server_poll": (st, [p, ctypes.POINTER(ctypes.c_uint32)]),
        "dialsort_server_drain": (st, [p]),
        "dialsort_server_info": (st, [p, u64, ctypes.POINTER(dialsort_request_info)]),
        "dialsort_server_release": (st, [p, u64]),
        "dialsort_status_sync": (st, [p, p]),
        "dialsort_result_total": (st, [p, p, ctypes.POINTER(u64)]),
        "dialsort_strerror": (ctypes.c_char_p, [st]),
        "dialsort_last_hip_error": (ctypes.c_int, []),
        "dialsort_set_launch_events": (st, [p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
        "dialsort_launch_name": (ctypes.c_char_p, [ctypes.c_uint32]),
        "dialsort_query_frequency": (st, [p, u64, p, u64, p, p]),
        "dialsort_query_presence": (st, [p, u64, p, u64, p, p]),
        "dialsort_prefix_workspace_bytes": (sz, [u64]),
        "dialsort_prefix": (st, [p, u64, p, p, sz, p]),
        "dialsort_query_range_count": (st, [p, u64, p, p, u64, p, p]),
        "dialsort_query_select": (st, [p, u64, p, u64, p, p]),
        "dialsort_sort_noalloc": (st, [p, u64, u64, p, p, p, p]),
        "dialsort_radix_workspace_bytes": (sz, [u64]),
        "dialsort_sort_radix": (st, [p, u64, ctypes.c_int, p, p, sz, p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    return lib


_lib = _load()
EXPORTED = ("dialsort_workspace_bytes", "dialsort_histogram", "dialsort_histogram_accumulate",
            "dialsort_histogram_offset", "dialsort_sort_offset", "dialsort_sort_lut", "dialsort_key_range",
            "dialsort_windows_workspace_bytes", "dialsort_sort_windows",
            "dialsort_reconstruct", "dialsort_sort",
            "dialsort_batched_workspace_bytes", "dialsort_sort_batched", "dialsort_sort_each",
            "dialsort_batch_prepare", "dialsort_batch_launch", "dialsort_batch_autotune",
            "dialsort_batch_default_config", "dialsort_batch_times", "dialsort_server_footprint", "dialsort_server_now_ms",
            "dialsort_server_create", "dialsort_server_destroy", "dialsort_server_submit", "dialsort_server_poll",
            "dialsort_server_drain", "dialsort_server_info", "dialsort_server_release", "dialsort_status_sync",
            "dialsort_result_total", "dialsort_strerror", "dialsort_last_hip_error",
            "dialsort_set_launch_events", "dialsort_launch_name", "dialsort_query_frequency",
            "dialsort_query_presence", "dialsort_prefix_workspace_bytes", "dialsort_prefix",
            "dialsort_query_range_count", "dialsort_query_select", "dialsort_radix_workspace_bytes",
            "dialsort_sort_radix", "dialsort_sort_noalloc")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.numel() and not t.is_cuda:
        raise ValueError("dialsort tensors must live on the GPU")
    if t.numel() and not t.is_contiguous():
        raise ValueError("dialsort tensors must be contiguous")
    return t.data_ptr() if t.numel() else None


def _w(size: int, *ts) -> bool:
    """True when every given tensor (None skipped) has elements of `size` bytes."""
    return all(t is None or t.element_size() == size for t in ts)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream or None
    return getattr(stream, "cuda_stream", stream) or None


def check(status: int) -> None:
    if status != DIALSORT_OK:
        raise DialSortError(status)


def dialsort_strerror(status: int) -> str:
    return _lib.dialsort_strerror(status).decode()


def dialsort_last_hip_error() -> int:
    return _lib.dialsort_last_hip_error()


def dialsort_workspace_bytes(n: int, U: int, mode: int) -> int:
    return _lib.dialsort_workspace_bytes(n, U, mode)


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """A device byte tensor usable as a workspace of at least nbytes."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def dialsort_histogram(keys: torch.Tensor, U: int, H: torch.Tensor, ws: torch.Tensor, stream=None) -> int:
    if not _w(4, keys, H) or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_histogram(_ptr(keys), keys.numel(), U, _ptr(H), _ptr(ws), ws.numel(), _stream(stream))


def dialsort_histogram_accumulate(keys: torch.Tensor, U: int, H: torch.Tensor, ws: torch.Tensor,
                                  stream=None) -> int:
    if not _w(4, keys, H) or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_histogram_accumulate(_ptr(keys), keys.numel(), U, _ptr(H), _ptr(ws), ws.numel(),
                                              _stream(stream))


def dialsort_histogram_offset(keys: torch.Tensor, lo: int, U: int, H: torch.Tensor, ws: torch.Tensor,
                              stream=None) -> int:
    if not _w(4, keys, H) or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_histogram_offset(_ptr(keys), keys.numel(), lo & 0xFFFFFFFF, U, _ptr(H), _ptr(ws),
                                          ws.numel(), _stream(stream))


def dialsort_sort_offset(keys: torch.Tensor, lo: int, U: int, H: torch.Tensor, out: torch.Tensor,
                         ws: torch.Tensor, stream=None) -> int:
    """Keys in [lo, lo + U) (mod 2^32); lo may be given as a signed int32."""
    if not _w(4, keys, H, out) or out.numel() < keys.numel() or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_sort_offset(_ptr(keys), keys.numel(), lo & 0xFFFFFFFF, U, _ptr(H), _ptr(out), _ptr(ws),
                                     ws.numel(), _stream(stream))


def dialsort_sort_lut(keys: torch.Tensor, U: int, lut: torch.Tensor, H: torch.Tensor, out: torch.Tensor,
                      ws: torch.Tensor, stream=None) -> int:
    """Indices in [0, U); out receives lut[k] for the indices in order."""
    if not _w(4, keys, H, out, lut) or out.numel() < keys.numel() or lut.numel() < U or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_sort_lut(_ptr(keys), keys.numel(), U, _ptr(lut), _ptr(H), _ptr(out), _ptr(ws), ws.numel(),
                                  _stream(stream))


def dialsort_windows_workspace_bytes(window_n: int, U: int) -> int:
    return _lib.dialsort_windows_workspace_bytes(window_n, U)


def dialsort_sort_windows(keys: torch.Tensor, window_n: int, count: int, U: int, H: torch.Tensor, out: torch.Tensor,
                          ws: torch.Tensor, ingest_stream=None, project_stream=None) -> int:
    """Tumbling windows of window_n keys: window w's ingestion on ingest_stream
    overlaps window w - 1's projection on project_stream.  H holds 2U counters."""
    if not _w(4, keys, H, out) or keys.numel() < window_n * count or out.numel() < window_n * count \
            or H.numel() < 2 * U:
        return DIALSORT_EINVAL
    return _lib.dialsort_sort_windows(_ptr(keys), window_n, count, U, _ptr(H), _ptr(out), _ptr(ws), ws.numel(),
                                      _stream(ingest_stream), _stream(project_stream))


def dialsort_key_range(keys: torch.Tensor, minmax: torch.Tensor, is_signed: bool = False, stream=None) -> int:
    """minmax[0] = min, minmax[1] = max of the keys (two 32-bit device words)."""
    if not _w(4, keys) or minmax.numel() * minmax.element_size() < 8:
        return DIALSORT_EINVAL
    return _lib.dialsort_key_range(_ptr(keys), keys.numel(), int(bool(is_signed)), _ptr(minmax), _stream(stream))


def dialsort_sort(keys: torch.Tensor, U: int, H: torch.Tensor, out: torch.Tensor, ws: torch.Tensor,
                  stream=None) -> int:
    if not _w(4, keys, H, out) or out.numel() < keys.numel() or H.numel() < U:
        return DIALSORT_EINVAL
    return _lib.dialsort_sort(_ptr(keys), keys.numel(), U, _ptr(H), _ptr(out), _ptr(ws), ws.numel(),
                              _stream(stream))


def dialsort_sort_noalloc(keys: torch.Tensor, U: int, H: torch.Tensor, out: torch.Tensor,
                          status: Optional[torch.Tensor] = None, stream=None) -> int:
    """dialsort_sort with the library's own per-device workspace (nothing is
    allocated); status: an optional one-word device tensor for the status word."""
    if not _w(4, keys, H, out, status) or out.numel() < keys.numel() or H.numel() < U:
        return DIALSORT_EINVAL
    if status is not None and status.numel() < 1:
        return DIALSORT_EINVAL
    return _lib.dialsort_sort_noalloc(_ptr(keys), keys.numel(), U, _ptr(H), _ptr(out), _ptr(status),
                                      _stream(stream))


def dialsort_reconstruct(H: torch.Tensor, out: torch.Tensor, ws: torch.Tensor, out_cap: Optional[int] = None,
                         stream=None) -> int:
    cap = out.numel() if out_cap is None else int(out_cap)
    if not _w(4, H, out) or cap > out.numel():
        return DIALSORT_EINVAL
    return _lib.dialsort_reconstruct(_ptr(H), H.numel(), _ptr(out), cap, _ptr(ws), ws.numel(), _stream(stream))


def make_descs(arrays: Sequence[Tuple[torch.Tensor, int, torch.Tensor, torch.Tensor]]):
    """(keys, U, H, out) tuples -> a ctypes array of dialsort_desc.  Raises
    DialSortError(DIALSORT_EINVAL) for keys, H or out without 4-byte elements,
    an H shorter than U or an out shorter than the keys."""
    descs = (dialsort_desc * max(len(arrays), 1))()
    for i, (k, U, H, o) in enumerate(arrays):
        if not _w(4, k, H, o) or H.numel() < U or o.numel() < k.numel():
            raise DialSortError(DIALSORT_EINVAL)
        descs[i] = dialsort_desc(_ptr(k), k.numel(), U, _ptr(H), _ptr(o))
    return descs


def dialsort_batched_workspace_bytes(descs, count: int) -> int:
    return _lib.dialsort_batched_workspace_bytes(descs, count)


def dialsort_sort_batched(descs, count: int, ws: torch.Tensor, stream=None) -> int:
    return _lib.dialsort_sort_batched(descs, count, _ptr(ws), ws.numel(), _stream(stream))


def dialsort_sort_each(descs, count: int, ws: torch.Tensor, stream=None) -> int:
    return _lib.dialsort_sort_each(descs, count, _ptr(ws), ws.numel(), _stream(stream))


def batch_config(block: int, log2_width: int, chunk_keys: int) -> dialsort_batch_config:
    return dialsort_batch_config(block, log2_width, chunk_keys)


def dialsort_batch_prepare(descs, count: int, config: Optional[dialsort_batch_config], ws: torch.Tensor,
                           stream=None) -> Tuple[int, dialsort_batch_plan]:
    plan = dialsort_batch_plan()
    cfg = ctypes.byref(config) if config is not None else None
    st = _lib.dialsort_batch_prepare(descs, count, cfg, _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(plan))
    return st, plan


def dialsort_batch_launch(plan: dialsort_batch_plan, stream=None) -> int:
    return _lib.dialsort_batch_launch(ctypes.byref(plan), _stream(stream))


def dialsort_batch_autotune(descs, count: int, ws: torch.Tensor, stream=None) -> Tuple[int, dialsort_batch_config]:
    best = dialsort_batch_config()
    st = _lib.dialsort_batch_autotune(descs, count, _ptr(ws), ws.numel(), _stream(stream), ctypes.byref(best))
    return st, best


def dialsort_batch_default_config(descs, count: int) -> Tuple[int, dialsort_batch_config]:
    cfg = dialsort_batch_config()
    st = _lib.dialsort_batch_default_config(descs, count, ctypes.byref(cfg))
    return st, cfg


UNIT_TYPES = ("hist", "partition", "rows", "bucket", "fill", "fill_late")


def dialsort_batch_times(plan: dialsort_batch_plan, count: int, stream=None, units: bool = False):
    """(status, per-array completion times in ms, whole-launch time in ms) of the
    last launch of `plan`; with units=True a fourth element maps every unit type
    to its (busy, waiting) workgroup-milliseconds."""
    arr = (ctypes.c_double * max(count, 1))()
    tot = ctypes.c_double(0.0)
    um = (ctypes.c_double * 12)()
    st = _lib.dialsort_batch_times(ctypes.byref(plan), _stream(stream), arr, count, ctypes.byref(tot), um)
    if units:
        return st, list(arr[:count]), tot.value, {t: (um[2 * i], um[2 * i + 1]) for i, t in enumerate(UNIT_TYPES)}
    return st, list(arr[:count]), tot.value


def dialsort_server_footprint(n: int, U: int) -> int:
    return _lib.dialsort_server_footprint(n, U)


def server_config(batch: dialsort_batch_config, max_inflight: int = 2, max_batch: int = 256) -> dialsort_server_config:
    return dialsort_server_config(batch, max_inflight, max_batch)


def dialsort_server_create(arena: torch.Tensor, config: dialsort_server_config) -> Tuple[int, Optional[int]]:
    h = ctypes.c_void_p()
    st = _lib.dialsort_server_create(_ptr(arena), arena.numel() * arena.element_size(), ctypes.byref(config),
                                     ctypes.byref(h))
    return st, h.value


def dialsort_server_now_ms(server: int) -> float:
    return _lib.dialsort_server_now_ms(server)


def dialsort_server_destroy(server: int) -> int:
    return _lib.dialsort_server_destroy(server)


def dialsort_server_submit(server: int, keys: torch.Tensor, U: int) -> Tuple[int, int]:
    rid = ctypes.c_uint64(0)
    if not _w(4, keys):
        return DIALSORT_EINVAL, 0
    st = _lib.dialsort_server_submit(server, _ptr(keys), keys.numel(), U, ctypes.byref(rid))
    return st, rid.value


def dialsort_server_poll(server: int) -> Tuple[int, int]:
    pending = ctypes.c_uint32(0)
    st = _lib.dialsort_server_poll(server, ctypes.byref(pending))
    return st, pending.value


def dialsort_server_drain(server: int) -> int:
    return _lib.dialsort_server_drain(server)


def dialsort_server_info(server: int, rid: int) -> Tuple[int, dialsort_request_info]:
    info = dialsort_request_info()
    st = _lib.dialsort_server_info(server, rid, ctypes.byref(info))
    return st, info


def dialsort_server_release(server: int, rid: int) -> int:
    return _lib.dialsort_server_release(server, rid)


def arena_view(arena: torch.Tensor, ptr: int, count: int) -> torch.Tensor:
    """The int32 view of `count` uint32 values at device address ptr inside the
    byte tensor `arena` (a request's H or output in a server arena)."""
    off = int(ptr) - arena.data_ptr()
    if count == 0:
        return arena[:0].view(torch.int32)
    if off < 0 or off % 4 or off + 4 * count > arena.numel():
        raise ValueError("address outside the arena")
    return arena[off:off + 4 * count].view(torch.int32)


def dialsort_status_sync(ws: torch.Tensor, stream=None) -> int:
    return _lib.dialsort_status_sync(_ptr(ws), _stream(stream))


def dialsort_result_total(ws: torch.Tensor, stream=None) -> Tuple[int, int]:
    total = ctypes.c_uint64(0)
    st = _lib.dialsort_result_total(_ptr(ws), _stream(stream), ctypes.byref(total))
    return st, total.value


def dialsort_set_launch_events(events, cap: int, count) -> int:
    """events: a ctypes array of hipEvent_t handles (or None to switch off);
    count: a ctypes.c_uint32 that receives the number of launches per call."""
    return _lib.dialsort_set_launch_events(events, cap, ctypes.byref(count) if count is not None else None)


def dialsort_launch_name(i: int) -> Optional[str]:
    r = _lib.dialsort_launch_name(i)
    return r.decode() if r else None


# ---- queries on H (frequency, presence, range-count, prefix, select) ----------


def dialsort_query_frequency(H: torch.Tensor, U: int, q: torch.Tensor, out: torch.Tensor, stream=None) -> int:
    if not _w(4, H, q, out) or H.numel() < U or out.numel() < q.numel():
        return DIALSORT_EINVAL
    return _lib.dialsort_query_frequency(_ptr(H), U, _ptr(q), q.numel(), _ptr(out), _stream(stream))


def dialsort_query_presence(H: torch.Tensor, U: int, q: torch.Tensor, out: torch.Tensor, stream=None) -> int:
    if not _w(4, H, q) or H.numel() < U or out.numel() < q.numel() or out.element_size() != 1:
        return DIALSORT_EINVAL
    return _lib.dialsort_query_presence(_ptr(H), U, _ptr(q), q.numel(), _ptr(out), _stream(stream))


def dialsort_prefix_workspace_bytes(U: int) -> int:
    return _lib.dialsort_prefix_workspace_bytes(U)


def dialsort_prefix(H: torch.Tensor, U: int, P: torch.Tensor, ws: torch.Tensor, stream=None) -> int:
    if not _w(4, H) or H.numel() < U or P.numel() < U + 1 or P.element_size() != 8:
        return DIALSORT_EINVAL
    return _lib.dialsort_prefix(_ptr(H), U, _ptr(P), _ptr(ws), ws.numel(), _stream(stream))


def dialsort_query_range_count(P: torch.Tensor, U: int, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor,
                               stream=None) -> int:
    if not _w(8, P, a, b, out) or P.numel() < U + 1 or b.numel() != a.numel() or out.numel() < a.numel():
        return DIALSORT_EINVAL
    return _lib.dialsort_query_range_count(_ptr(P), U, _ptr(a), _ptr(b), a.numel(), _ptr(out), _stream(stream))


def dialsort_query_select(P: torch.Tensor, U: int, r: torch.Tensor, out: torch.Tensor, stream=None) -> int:
    if not _w(8, P, r) or not _w(4, out) or P.numel() < U + 1 or out.numel() < r.numel():
        return DIALSORT_EINVAL
    return _lib.dialsort_query_select(_ptr(P), U, _ptr(r), r.numel(), _ptr(out), _stream(stream))


# ---- DialSort-Radix (the whole 32-bit range) ------------------------------------


def dialsort_radix_workspace_bytes(n: int) -> int:
    return _lib.dialsort_radix_workspace_bytes(n)


def dialsort_sort_radix(keys: torch.Tensor, out: torch.Tensor, ws: torch.Tensor, is_signed: bool = False,
                        stream=None) -> int:
    if not _w(4, keys, out) or out.numel() < keys.numel():
        return DIALSORT_EINVAL
    return _lib.dialsort_sort_radix(_ptr(keys), keys.numel(), 1 if is_signed else 0, _ptr(out), _ptr(ws),
                                    ws.numel(), _stream(stream))
