"""DialSort CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never does, and shares no code with it.

``dialsort_oracle.c`` states the method as the paper defines it: ingestion,
Eq. (1) (Sec. 3.3), then the ordered projection, Eq. (2) (Sec. 3.3), and the
sort over a universe that starts anywhere (phi of Sec. 3.4), the sort of a
domain given by its index map with phi^-1 as a table and the key range that
fixes the smallest offset map (both Sec. 3.4), DialSort-Radix (Sec. 8, full
int32 range), and the
queries that read H directly (frequency, presence and range-count, from the
paragraph on the canonical ordered state in Sec. 3.3; prefix and select, the
running count and the projection read at one position).  This
module compiles that file with gcc (``build()``), loads it with ctypes and
marshals numpy arrays.  ``crn.py`` holds the Conflict Resolution Network model of
Sec. 6, used by tests only.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

OK, EINVAL, ERANGE, EOVERFLOW = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dialsort_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib: Optional[ctypes.CDLL] = None


def build() -> str:
    """Compile the C oracle into oracle/liboracle.so (plain gcc, -O2), and the
    CPU-parallel benchmark baseline beside it (oracle/cpu_parallel.py)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                           _SRC, "-o", tmp])
    os.replace(tmp, _LIB_PATH)
    from . import cpu_parallel

    cpu_parallel.build()
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.oracle_histogram.argtypes = [p, u64, u64, p]
        lib.oracle_histogram.restype = ctypes.c_int
        lib.oracle_reconstruct.argtypes = [p, u64, p, u64, ctypes.POINTER(u64)]
        lib.oracle_reconstruct.restype = ctypes.c_int
        lib.oracle_sort.argtypes = [p, u64, u64, p, p]
        lib.oracle_sort.restype = ctypes.c_int
        lib.oracle_histogram_accumulate.argtypes = [p, u64, u64, p]
        lib.oracle_histogram_accumulate.restype = ctypes.c_int
        lib.oracle_sort_offset.argtypes = [p, u64, ctypes.c_uint32, u64, p, p]
        lib.oracle_sort_offset.restype = ctypes.c_int
        lib.oracle_sort_radix.argtypes = [p, u64, ctypes.c_int, p, p]
        lib.oracle_sort_radix.restype = ctypes.c_int
        lib.oracle_sort_lut.argtypes = [p, u64, u64, p, p, p]
        lib.oracle_sort_lut.restype = ctypes.c_int
        lib.oracle_key_range.argtypes = [p, u64, ctypes.c_int, p]
        lib.oracle_key_range.restype = ctypes.c_int
        for name in ("oracle_frequency", "oracle_presence"):
            getattr(lib, name).argtypes = [p, u64, p, u64, p]
            getattr(lib, name).restype = None
        lib.oracle_range_count.argtypes = [p, u64, p, p, u64, p]
        lib.oracle_range_count.restype = None
        lib.oracle_prefix.argtypes = [p, u64, p]
        lib.oracle_prefix.restype = None
        lib.oracle_select.argtypes = [p, u64, p, u64, p]
        lib.oracle_select.restype = None
        _lib = lib
    return _lib


def _as_u32(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype == np.int32:
        a = a.view(np.uint32)
    if a.dtype != np.uint32:
        a = a.astype(np.uint32)
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def histogram(keys, U: int) -> Tuple[int, np.ndarray]:
    """Eq. (1): returns (status, H) with H of length U (uint32)."""
    k = _as_u32(keys)
    H = np.zeros(U, dtype=np.uint32)
    st = _load().oracle_histogram(_ptr(k), k.size, U, H.ctypes.data_as(ctypes.c_void_p))
    return st, H


def histogram_accumulate(keys, U: int, H) -> Tuple[int, np.ndarray]:
    """Eq. (1) over one more piece of a key stream: returns (status, H + counts)."""
    k = _as_u32(keys)
    h = _as_u32(H).copy()
    assert h.size == U
    st = _load().oracle_histogram_accumulate(_ptr(k), k.size, U, h.ctypes.data_as(ctypes.c_void_p))
    return st, h


def sort_offset(keys, lo: int, U: int) -> Tuple[int, np.ndarray, np.ndarray]:
    """Sec. 3.4 with phi(x) = x - lo (mod 2^32): returns (status, H, out)."""
    k = _as_u32(keys)
    H = np.zeros(U, dtype=np.uint32)
    out = np.empty_like(k)
    st = _load().oracle_sort_offset(_ptr(k), k.size, lo & 0xFFFFFFFF, U, H.ctypes.data_as(ctypes.c_void_p),
                                    _ptr(out))
    return st, H, out


def sort_lut(keys, U: int, lut) -> Tuple[int, np.ndarray, np.ndarray]:
    """Sec. 3.4 with phi^-1 as a table: indices in [0, U), out = lut[k] per
    index in ascending k.  Returns (status, H, out)."""
    k = _as_u32(keys)
    t = _as_u32(lut)
    if t.size < U:
        return EINVAL, None, None
    H = np.zeros(U, dtype=np.uint32)
    out = np.empty(max(k.size, 1), dtype=np.uint32)
    st = _load().oracle_sort_lut(_ptr(k), k.size, U, _ptr(t), H.ctypes.data_as(ctypes.c_void_p), _ptr(out))
    return st, H, out[: k.size]


def key_range(keys, is_signed: bool = False) -> Tuple[int, int, int]:
    """(status, min, max) as uint32 bit patterns (compared as int32 when signed)."""
    k = _as_u32(keys)
    mm = np.zeros(2, dtype=np.uint32)
    st = _load().oracle_key_range(_ptr(k), k.size, 1 if is_signed else 0, _ptr(mm))
    return st, int(mm[0]), int(mm[1])


def sort_radix(keys, is_signed: bool = False) -> Tuple[int, np.ndarray]:
    """DialSort-Radix: LSD base 256, 4 passes (signed: sign bit flipped)."""
    k = _as_u32(keys)
    out = np.empty(max(k.size, 1), dtype=np.uint32)
    tmp = np.empty(max(k.size, 1), dtype=np.uint32)
    st = _load().oracle_sort_radix(_ptr(k), k.size, 1 if is_signed else 0, _ptr(out), _ptr(tmp))
    return st, out[: k.size]


def reconstruct(H, out_cap: Optional[int] = None) -> Tuple[int, np.ndarray]:
    """Eq. (2): returns (status, out) where out holds min(sum H, out_cap) keys."""
    h = _as_u32(H)
    total = int(h.sum(dtype=np.uint64))
    cap = total if out_cap is None else int(out_cap)
    # the C routine never writes more than min(cap, total) elements; keep the
    # buffer non-empty so that a nonzero cap never comes with a null pointer
    out = np.empty(max(min(cap, total), 1), dtype=np.uint32)
    written = ctypes.c_uint64(0)
    st = _load().oracle_reconstruct(h.ctypes.data_as(ctypes.c_void_p), h.size,
                                    _ptr(out), cap, ctypes.byref(written))
    return st, out[: written.value]


def sort(keys, U: int, in_place: bool = False) -> Tuple[int, np.ndarray, np.ndarray]:
    """Eq. (1) then Eq. (2): returns (status, H, out).  With in_place=True the
    projection is written over (a copy of) the key array, as in Sec. 9.2."""
    k = _as_u32(keys).copy()
    H = np.zeros(U, dtype=np.uint32)
    out = k if in_place else np.empty_like(k)
    st = _load().oracle_sort(_ptr(k), k.size, U, H.ctypes.data_as(ctypes.c_void_p), _ptr(out))
    return st, H, out


# ---- queries on H (Sec. 3.3, the paragraph on the canonical ordered state) ----


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def frequency(H, q) -> np.ndarray:
    """H[k] for every query key k (0 outside [0, U))."""
    h, qq = _as_u32(H), _as_u32(q)
    out = np.zeros(max(qq.size, 1), dtype=np.uint32)
    _load().oracle_frequency(_ptr(h), h.size, _ptr(qq), qq.size, _ptr(out))
    return out[: qq.size]


def presence(H, q) -> np.ndarray:
    """1 where the query key occurs (H[k] > 0), else 0 (uint8)."""
    h, qq = _as_u32(H), _as_u32(q)
    out = np.zeros(max(qq.size, 1), dtype=np.uint8)
    _load().oracle_presence(_ptr(h), h.size, _ptr(qq), qq.size, _ptr(out))
    return out[: qq.size]


def range_count(H, a, b) -> np.ndarray:
    """Keys in [a, b) for every query, bounds cut at U (uint64)."""
    h, aa, bb = _as_u32(H), _u64(a), _u64(b)
    out = np.zeros(max(aa.size, 1), dtype=np.uint64)
    _load().oracle_range_count(_ptr(h), h.size, _ptr(aa), _ptr(bb), aa.size, _ptr(out))
    return out[: aa.size]


def prefix(H) -> np.ndarray:
    """P[k] = H[0] + ... + H[k-1], k = 0 .. U (uint64, U + 1 entries)."""
    h = _as_u32(H)
    P = np.zeros(h.size + 1, dtype=np.uint64)
    _load().oracle_prefix(_ptr(h), h.size, _ptr(P))
    return P


def select(H, r) -> np.ndarray:
    """The element at position r of the ordered projection (0xFFFFFFFF past the end)."""
    h, rr = _as_u32(H), _u64(r)
    out = np.zeros(max(rr.size, 1), dtype=np.uint32)
    _load().oracle_select(_ptr(h), h.size, _ptr(rr), rr.size, _ptr(out))
    return out[: rr.size]
