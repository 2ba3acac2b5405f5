"""GPU parity of accumulating ingestion (a key stream ingested piece by piece
into one resident H, then projected once), against the oracle's own
piece-by-piece ingestion of the same seeded pieces."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


def dev_u32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(DEV)


@pytest.mark.parametrize("U,sizes", [
    (1000, [0, 1, 7, 5000, 123456]),                # LDS path, pieces from empty to large
    (65536, [1 << 20, 3, 999999, 1 << 18]),         # packed LDS path
    ((1 << 20) + 3, [5000, 2_000_000, 70000]),      # global and partitioned paths
    (1 << 24, [10_000_000, 3_000_000, 17]),         # the large universe
])
def test_stream_equals_whole(ds, U, sizes):
    say(f"stream U={U} pieces={sizes}")
    rng = np.random.default_rng(U + len(sizes))
    pieces = [rng.integers(0, U, m).astype(np.uint32) for m in sizes]
    H = torch.zeros(U, dtype=torch.int32, device=DEV)
    H_ref = np.zeros(U, dtype=np.uint32)
    for p in pieces:
        ws = ds.workspace(ds.dialsort_workspace_bytes(p.size, U, ds.DIALSORT_MODE_ACCUMULATE))
        ds.check(ds.dialsort_histogram_accumulate(dev_u32(p), U, H, ws))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
        st, H_ref = oracle.histogram_accumulate(p, U, H_ref)
        assert st == oracle.OK
        assert np.array_equal(w.as_u32(H), H_ref)
    # the projection of the accumulated state is the sort of the whole stream
    whole = np.concatenate(pieces)
    n = whole.size
    out = torch.empty(max(n, 1), dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_RECONSTRUCT))
    ds.check(ds.dialsort_reconstruct(H, out[:n], ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    st, _, out_ref = oracle.sort(whole, U)
    assert np.array_equal(w.as_u32(out[:n]), out_ref)


def test_accumulate_overflow_and_range(ds):
    U = 4096
    H0 = np.zeros(U, dtype=np.uint32)
    H0[7] = 0xFFFFFFF0
    H = dev_u32(H0)
    keys = np.full(100, 7, dtype=np.uint32)
    ws = ds.workspace(ds.dialsort_workspace_bytes(keys.size, U, ds.DIALSORT_MODE_ACCUMULATE))
    say("a bin passing 2^32 - 1")
    ds.check(ds.dialsort_histogram_accumulate(dev_u32(keys), U, H, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_EOVERFLOW
    st, _ = oracle.histogram_accumulate(keys, U, H0)
    assert st == oracle.EOVERFLOW
    say("a key past the universe")
    H = torch.zeros(U, dtype=torch.int32, device=DEV)
    bad = np.array([1, 2, U], dtype=np.uint32)
    ds.check(ds.dialsort_histogram_accumulate(dev_u32(bad), U, H, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_ERANGE
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    assert ds.dialsort_histogram_accumulate(dev_u32(keys), U, H, small) == ds.DIALSORT_EWORKSPACE
