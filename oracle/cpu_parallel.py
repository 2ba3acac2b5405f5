"""CPU-parallel DialSort baseline -- TEST AND BENCHMARK INFRASTRUCTURE ONLY.

Only ``tests/`` and the CPU-baseline leg of ``bench.py`` use this module.  It
wraps ``cpu_parallel.c`` (private per-thread histograms of Eq. (1), a merge,
and the projection of Eq. (2) by ranges of bins in parallel), which gives a
multi-core host timing beside the GPU path.  It is not the oracle: the tests
check its output against the oracle.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_parallel.c")
_LIB_PATH = os.path.join(_HERE, "libcpupar.so")
_lib: Optional[ctypes.CDLL] = None


def build() -> str:
    """Compile cpu_parallel.c into oracle/libcpupar.so (gcc -O2 -pthread)."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                           _SRC, "-o", tmp])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, p = ctypes.c_uint64, ctypes.c_void_p
        lib.cpu_parallel_sort.argtypes = [p, u64, u64, p, p, ctypes.c_int]
        lib.cpu_parallel_sort.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    """The host threads this process may use: OMP_NUM_THREADS if set, else the
    CPUs it may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def sort(keys: np.ndarray, U: int, nthreads: Optional[int] = None, out: bool = True
         ) -> Tuple[int, np.ndarray, Optional[np.ndarray]]:
    """Returns (status, H, out): status 0 ok, 1 bad arguments, 2 a key >= U."""
    k = np.ascontiguousarray(keys).view(np.uint32)
    H = np.empty(U, dtype=np.uint32)
    o = np.empty(max(k.size, 1), dtype=np.uint32) if out else None
    st = _load().cpu_parallel_sort(k.ctypes.data_as(ctypes.c_void_p), k.size, U, H.ctypes.data_as(ctypes.c_void_p),
                                   o.ctypes.data_as(ctypes.c_void_p) if o is not None else None,
                                   int(nthreads or default_threads()))
    return st, H, (o[: k.size] if o is not None else None)
