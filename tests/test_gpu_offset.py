"""GPU parity of sorting over a universe that starts at lo (the order-
isomorphism phi(x) = x - lo of Sec. 3.4): signed int32 keys and universes that
wrap past 2^32 - 1, on every path kind, against the oracle's offset sort."""

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


def run(ds, keys_u32, lo, U):
    n = keys_u32.size
    kd = torch.from_numpy(keys_u32.view(np.int32)).to(DEV)
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = torch.empty(max(n, 1), dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT))
    ds.check(ds.dialsort_sort_offset(kd, lo, U, H, out[:n], ws))
    st_dev = ds.dialsort_status_sync(ws)
    st, H_ref, out_ref = oracle.sort_offset(keys_u32, lo, U)
    return st_dev, st, w.as_u32(H), H_ref, w.as_u32(out[:n]), out_ref, kd, ws


@pytest.mark.parametrize("lo,U,n", [
    (-1000, 2001, 50000),                      # signed, LDS path
    (-(1 << 15), 1 << 16, 1 << 20),            # signed, packed LDS path
    (-(1 << 23), 1 << 24, 5_000_000),          # signed, partitioned path
    (-(1 << 19), 1 << 20, 3000),               # signed, global-atomics path (few keys, large U)
    (0xFFFFFF00, 512, 100000),                 # a universe that wraps past 2^32 - 1
    (123456789, 70001, 200000),
])
def test_offset_sort_matches_the_oracle(ds, lo, U, n):
    say(f"offset sort lo={lo} U={U} n={n}")
    rng = np.random.default_rng(abs(lo) % 1000 + U + n)
    keys = ((lo + rng.integers(0, U, n)) % 2**32).astype(np.uint32)
    st_dev, st, H, H_ref, out, out_ref, kd, ws = run(ds, keys, lo, U)
    assert st == oracle.OK and st_dev == ds.DIALSORT_OK
    assert np.array_equal(H, H_ref)
    assert np.array_equal(out, out_ref)
    # histogram-only form
    Hd = torch.empty(U, dtype=torch.int32, device=DEV)
    wsh = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_HISTOGRAM))
    ds.check(ds.dialsort_histogram_offset(kd, lo, U, Hd, wsh))
    assert ds.dialsort_status_sync(wsh) == ds.DIALSORT_OK
    assert np.array_equal(w.as_u32(Hd), H_ref)
    if lo < 0:  # signed keys: numpy's signed order
        assert np.array_equal(out.view(np.int32), np.sort(keys.view(np.int32)))


def test_offset_out_of_range(ds):
    lo, U = -50, 100
    keys = np.array([-50, 49, 0, 50], dtype=np.int32).view(np.uint32)
    say("a key past lo + U")
    st_dev, st, *_ = run(ds, keys, lo, U)
    assert st == oracle.ERANGE and st_dev == ds.DIALSORT_ERANGE
    keys = np.array([-51, 0], dtype=np.int32).view(np.uint32)
    say("a key below lo")
    st_dev, st, *_ = run(ds, keys, lo, U)
    assert st == oracle.ERANGE and st_dev == ds.DIALSORT_ERANGE
