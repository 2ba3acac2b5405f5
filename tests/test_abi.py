"""The C-ABI library without a GPU: it loads, exports every symbol declared in
include/dialsort.h, and rejects bad arguments on the host before anything is
enqueued (those paths make no HIP call)."""

from __future__ import annotations

import ctypes
import os
import re

import pytest

import paper_2605_16667_amd as ds

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dialsort.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dialsort_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(ds.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(ds.EXPORTED) == names


def test_workspace_query():
    assert ds.dialsort_workspace_bytes(10, 0, 1) == 0
    assert ds.dialsort_workspace_bytes(10, (1 << 32) + 1, 1) == 0
    for n, U in [(0, 1), (1, 1), (1 << 20, 1 << 16), (10**8, 1 << 24), (1 << 28, 1 << 16), (5, 1 << 32)]:
        for mode in (0, 1, 2):
            assert ds.dialsort_workspace_bytes(n, U, mode) >= 512


FAKE = 0x100000  # never dereferenced: every call below fails its host checks


def test_host_argument_checks():
    lib = ds._lib
    big = 1 << 40
    # U == 0 and U > 2^32
    assert lib.dialsort_histogram(FAKE, 4, 0, FAKE, FAKE, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort(FAKE, 4, (1 << 32) + 1, FAKE, FAKE, FAKE, big, None) == ds.DIALSORT_EINVAL
    # null H, null keys with n > 0
    assert lib.dialsort_histogram(FAKE, 4, 8, None, FAKE, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_histogram(None, 4, 8, FAKE, FAKE, big, None) == ds.DIALSORT_EINVAL
    # misaligned pointers
    assert lib.dialsort_sort(FAKE + 2, 4, 8, FAKE + 4096, FAKE + 8192, FAKE + 16384, big, None) == ds.DIALSORT_EINVAL
    # n beyond uint32 counters
    assert lib.dialsort_histogram(FAKE, 1 << 32, 8, FAKE, FAKE, big, None) == ds.DIALSORT_EOVERFLOW
    # workspace missing / too small
    assert lib.dialsort_histogram(FAKE, 4, 8, FAKE + 4096, None, big, None) == ds.DIALSORT_EWORKSPACE
    assert lib.dialsort_histogram(FAKE, 4, 8, FAKE + 4096, FAKE, 16, None) == ds.DIALSORT_EWORKSPACE
    # out partially overlapping keys; H overlapping keys
    assert lib.dialsort_sort(FAKE, 100, 8, FAKE + 4096, FAKE + 8, FAKE + 8192, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_histogram(FAKE, 100, 8, FAKE + 16, FAKE + 8192, big, None) == ds.DIALSORT_EINVAL
    # reconstruct: out_cap at or beyond 2^62, overlap with H
    assert lib.dialsort_reconstruct(FAKE, 8, FAKE + 4096, 1 << 62, FAKE, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_reconstruct(FAKE, 8, FAKE + 16, 4, FAKE + 8192, big, None) == ds.DIALSORT_EINVAL
    # lookup-table sort: null or misaligned table, table overlapping H or out
    assert lib.dialsort_sort_lut(FAKE, 4, 8, None, FAKE + 4096, FAKE + 8192, FAKE, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort_lut(FAKE, 4, 8, FAKE + 2, FAKE + 4096, FAKE + 8192, FAKE, big, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort_lut(FAKE, 4, 8, FAKE + 4100, FAKE + 4096, FAKE + 8192, FAKE, big,
                                 None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort_lut(FAKE, 4, 8, FAKE + 8200, FAKE + 4096, FAKE + 8192, FAKE, big,
                                 None) == ds.DIALSORT_EINVAL
    # tumbling windows: out overlapping keys, H overlapping out, window past 2^32 - 1 keys
    assert lib.dialsort_sort_windows(FAKE, 4, 2, 8, FAKE + 8192, FAKE + 16, FAKE + 16384, big, None,
                                     None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort_windows(FAKE, 4, 2, 8, FAKE + 4100, FAKE + 4096, FAKE + 16384, big, None,
                                     None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_sort_windows(FAKE, 1 << 32, 1, 8, FAKE + 8192, FAKE + 4096, FAKE + 16384, big, None,
                                     None) == ds.DIALSORT_EOVERFLOW
    assert lib.dialsort_windows_workspace_bytes(1 << 32, 8) == 0
    # key range: null result, keys missing, result overlapping the keys, n too large
    assert lib.dialsort_key_range(FAKE, 4, 0, None, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_key_range(None, 4, 0, FAKE, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_key_range(FAKE, 4, 0, FAKE + 8, None) == ds.DIALSORT_EINVAL
    assert lib.dialsort_key_range(FAKE, 1 << 32, 0, FAKE + 4096, None) == ds.DIALSORT_EOVERFLOW


def test_batched_argument_checks():
    d = (ds.dialsort_desc * 2)()
    d[0] = ds.dialsort_desc(FAKE, 4, 8, FAKE + 4096, FAKE + 8192)
    d[1] = ds.dialsort_desc(FAKE, 4, 0, FAKE + 4096, FAKE + 8192)  # U == 0
    assert ds._lib.dialsort_sort_batched(d, 2, FAKE + 65536, 1 << 40, None) == ds.DIALSORT_EINVAL
    assert ds._lib.dialsort_batched_workspace_bytes(d, 1) > 0


def test_batch_host_checks():
    d = (ds.dialsort_desc * 2)()
    d[0] = ds.dialsort_desc(FAKE, 4, 8, FAKE + 4096, FAKE + 8192)
    d[1] = ds.dialsort_desc(FAKE, 4, 1 << 32, FAKE + 4096 * 4, FAKE + 8192 * 4)
    # the second array is outside the fused form (U > 1024 * 2^16)
    assert ds._lib.dialsort_batched_workspace_bytes(d, 2) > 0
    plan = ds.dialsort_batch_plan()
    cfg = ds.batch_config(1024, 16, 1 << 20)
    assert ds._lib.dialsort_batch_prepare(d, 2, ctypes.byref(cfg), FAKE, 1 << 40, None,
                                          ctypes.byref(plan)) == ds.DIALSORT_EINVAL
    # bad configurations
    for bad in [ds.batch_config(256, 16, 1 << 20), ds.batch_config(1024, 13, 1 << 20),
                ds.batch_config(1024, 17, 1 << 20), ds.batch_config(1024, 16, 3 << 18),
                ds.batch_config(1024, 16, 1 << 23)]:
        assert ds._lib.dialsort_batch_prepare(d, 1, ctypes.byref(bad), FAKE, 1 << 40, None,
                                              ctypes.byref(plan)) == ds.DIALSORT_EINVAL
    # misaligned keys are outside the fused form
    d[0] = ds.dialsort_desc(FAKE + 4, 4, 8, FAKE + 4096, FAKE + 8192)
    assert ds._lib.dialsort_batch_prepare(d, 1, ctypes.byref(cfg), FAKE, 1 << 40, None,
                                          ctypes.byref(plan)) == ds.DIALSORT_EINVAL
    # null plan / launch of an empty plan
    assert ds._lib.dialsort_batch_prepare(d, 1, ctypes.byref(cfg), FAKE, 1 << 40, None, None) == ds.DIALSORT_EINVAL
    assert ds._lib.dialsort_batch_launch(ctypes.byref(ds.dialsort_batch_plan()), None) == ds.DIALSORT_EINVAL


def test_batched_workspace_covers_every_config():
    d = (ds.dialsort_desc * 3)()
    d[0] = ds.dialsort_desc(FAKE, 1 << 22, 1 << 20, FAKE, FAKE)
    d[1] = ds.dialsort_desc(FAKE, 1 << 20, 1 << 16, FAKE, FAKE)
    d[2] = ds.dialsort_desc(FAKE, 0, 1 << 10, FAKE, FAKE)
    b = ds._lib.dialsort_batched_workspace_bytes(d, 3)
    # at least the staging of the partitioned array (2 B per key) and the
    # partial rows of the LDS array at the smallest chunk (4 copies of U)
    assert b >= 2 * (1 << 22) + 4 * 4 * (1 << 16)


def test_server_host_checks():
    bad = ds.server_config(ds.batch_config(1024, 16, 1 << 20), 0, 8)  # max_inflight 0
    h = ctypes.c_void_p()
    assert ds._lib.dialsort_server_create(FAKE, 1 << 30, ctypes.byref(bad), ctypes.byref(h)) == ds.DIALSORT_EINVAL
    bad = ds.server_config(ds.batch_config(1024, 16, 1 << 20), 9, 8)
    assert ds._lib.dialsort_server_create(FAKE, 1 << 30, ctypes.byref(bad), ctypes.byref(h)) == ds.DIALSORT_EINVAL
    bad = ds.server_config(ds.batch_config(100, 16, 1 << 20), 2, 8)
    assert ds._lib.dialsort_server_create(FAKE, 1 << 30, ctypes.byref(bad), ctypes.byref(h)) == ds.DIALSORT_EINVAL
    assert ds._lib.dialsort_server_create(None, 1 << 30, ctypes.byref(bad), ctypes.byref(h)) == ds.DIALSORT_EINVAL
    rid = ctypes.c_uint64()
    assert ds._lib.dialsort_server_submit(None, FAKE, 4, 8, ctypes.byref(rid)) == ds.DIALSORT_EINVAL
    assert ds._lib.dialsort_server_poll(None, None) == ds.DIALSORT_EINVAL
    assert ds._lib.dialsort_server_destroy(None) == ds.DIALSORT_EINVAL
    # footprint: H and output, each rounded up to 256 bytes
    assert ds.dialsort_server_footprint(1000, 1 << 16) == (1 << 18) + 4096
    assert ds.dialsort_server_footprint(0, 1) == 512


def test_strerror():
    for s in range(6):
        assert ds.dialsort_strerror(s)


def test_binding_rejects_short_or_narrow_tensors():
    """The binding returns EINVAL before any call for H shorter than U, keys,
    H or out without 4-byte elements, and P / query arguments of the wrong
    width (CPU tensors: nothing reaches the library or the device)."""
    import torch

    k32 = torch.zeros(16, dtype=torch.int32)
    k16 = torch.zeros(16, dtype=torch.int16)
    k64 = torch.zeros(16, dtype=torch.int64)
    H = torch.zeros(64, dtype=torch.int32)
    ws = torch.zeros(16, dtype=torch.uint8)
    E = ds.DIALSORT_EINVAL
    U = 64
    for f in (ds.dialsort_histogram, ds.dialsort_histogram_accumulate):
        assert f(k32, U + 1, H, ws) == E            # H shorter than U
        assert f(k16, U, H, ws) == E                # 2-byte keys
        assert f(k32, U, H.view(torch.int16), ws) == E
    assert ds.dialsort_histogram_offset(k32, 0, U + 1, H, ws) == E
    assert ds.dialsort_histogram_offset(k64, 0, U, H, ws) == E
    out = torch.zeros(16, dtype=torch.int32)
    assert ds.dialsort_sort(k32, U + 1, H, out, ws) == E
    assert ds.dialsort_sort(k16, U, H, out, ws) == E
    assert ds.dialsort_sort(k32, U, H, out.view(torch.int16)[:16], ws) == E
    assert ds.dialsort_sort(k32, U, H, torch.zeros(8, dtype=torch.int32), ws) == E
    assert ds.dialsort_sort_offset(k32, 0, U + 1, H, out, ws) == E
    assert ds.dialsort_sort_offset(k64, 0, U, H, out, ws) == E
    lut = torch.zeros(U, dtype=torch.int32)
    assert ds.dialsort_sort_lut(k32, U, lut, torch.zeros(U - 1, dtype=torch.int32), out, ws) == E
    assert ds.dialsort_sort_lut(k32, U, lut.to(torch.int64), H, out, ws) == E
    assert ds.dialsort_sort_windows(k16, 8, 2, U, torch.zeros(2 * U, dtype=torch.int32), out, ws) == E
    assert ds.dialsort_key_range(k16, torch.zeros(2, dtype=torch.int32)) == E
    assert ds.dialsort_reconstruct(H.view(torch.int16), out, ws) == E
    assert ds.dialsort_reconstruct(H, out.to(torch.int64), ws) == E
    assert ds.dialsort_sort_radix(k16, out, ws) == E
    # queries: H width and length, P / a / b / r as 8-byte words
    q = torch.zeros(4, dtype=torch.int32)
    assert ds.dialsort_query_frequency(H, U + 1, q, q.clone()) == E
    assert ds.dialsort_query_frequency(H, U, q.to(torch.int16), q.clone()) == E
    assert ds.dialsort_query_presence(H[:U - 1], U, q, torch.zeros(4, dtype=torch.uint8)) == E
    P = torch.zeros(U + 1, dtype=torch.int64)
    assert ds.dialsort_prefix(H[:U - 1], U, P, ws) == E
    a = torch.zeros(4, dtype=torch.int64)
    assert ds.dialsort_query_range_count(P, U, a.to(torch.int32), a, a.clone()) == E
    assert ds.dialsort_query_range_count(P[:U], U, a, a, a.clone()) == E
    assert ds.dialsort_query_select(P, U, a.to(torch.int32), q) == E
    assert ds.dialsort_query_select(P, U, a, a.clone()) == E
    # the batched descriptor table refuses the same
    with pytest.raises(ds.DialSortError):
        ds.make_descs([(k32, U + 1, H, out)])
    with pytest.raises(ds.DialSortError):
        ds.make_descs([(k16, U, H, out)])
