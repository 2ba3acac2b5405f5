"""GPU parity of the other two forms of phi of Sec. 3.4: a domain given by its
index map with phi^-1 as a lookup table (dialsort_sort_lut, on every path
kind), and the key range that fixes the smallest offset map
(dialsort_key_range), against the oracle."""

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


def sort_lut(ds, keys_u32, U, lut_u32, in_place=False):
    n = keys_u32.size
    kd = torch.from_numpy(keys_u32.view(np.int32).copy()).to(DEV)
    lut = torch.from_numpy(lut_u32.view(np.int32).copy()).to(DEV)
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = kd if in_place else torch.empty(max(n, 1), dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT))
    ds.check(ds.dialsort_sort_lut(kd, U, lut, H, out[:n], ws))
    return ds.dialsort_status_sync(ws), w.as_u32(H), w.as_u32(out[:n])


@pytest.mark.parametrize("U,n", [
    (7, 1000),              # LDS path, tiny universe
    (2001, 50000),          # LDS path
    (1 << 16, 1 << 20),     # packed LDS path
    (1 << 24, 5_000_000),   # partitioned path
    (1 << 24, 20_000_000),  # partitioned path, an 80 MB output (non-temporal fill stores from 64 MiB)
    (1 << 20, 3000),        # global-atomics path (few keys, large U)
    (70001, 200_003),
])
@pytest.mark.parametrize("table", ["increasing", "permutation"])
def test_lut_sort_matches_the_oracle(ds, U, n, table):
    say(f"lut sort U={U} n={n} table={table}")
    rng = np.random.default_rng(U + n + len(table))
    keys = rng.integers(0, U, n).astype(np.uint32)
    if table == "increasing":
        lut = np.cumsum(rng.integers(1, 200, U, dtype=np.uint64)).astype(np.uint32)
    else:
        lut = rng.permutation(U).astype(np.uint32) ^ np.uint32(0xA5A50000)
    st_dev, H, out = sort_lut(ds, keys, U, lut)
    st, H_ref, out_ref = oracle.sort_lut(keys, U, lut)
    assert st == oracle.OK and st_dev == ds.DIALSORT_OK
    assert np.array_equal(H, H_ref)
    assert np.array_equal(out, out_ref)


def test_lut_sort_in_place_empty_and_errors(ds):
    rng = np.random.default_rng(5)
    U = 4096
    lut = rng.integers(0, 2**32, U, dtype=np.uint64).astype(np.uint32)
    keys = rng.integers(0, U, 300_001).astype(np.uint32)
    say("lut sort in place")
    st_dev, _, out = sort_lut(ds, keys, U, lut, in_place=True)
    assert st_dev == ds.DIALSORT_OK
    assert np.array_equal(out, oracle.sort_lut(keys, U, lut)[2])
    say("lut sort, no keys")
    st_dev, H, out = sort_lut(ds, np.array([], dtype=np.uint32), U, lut)
    assert st_dev == ds.DIALSORT_OK and out.size == 0 and not H.any()
    say("lut sort, an index past U")
    st_dev, _, _ = sort_lut(ds, np.array([0, U], dtype=np.uint32), U, lut)
    assert st_dev == ds.DIALSORT_ERANGE
    # the table may not overlap H or the output
    kd = torch.zeros(100, dtype=torch.int32, device=DEV)
    buf = torch.zeros(U + 100, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(100, U, ds.DIALSORT_MODE_SORT))
    assert ds.dialsort_sort_lut(kd, U, buf[:U], buf[:U], torch.empty_like(kd), ws) == ds.DIALSORT_EINVAL
    assert ds.dialsort_sort_lut(kd, U, buf[:U], torch.empty(U, dtype=torch.int32, device=DEV),
                                buf[U - 50:U + 50], ws) == ds.DIALSORT_EINVAL


@pytest.mark.parametrize("n", [0, 1, 2, 2047, 2049, 1_000_003, 50_000_000])
@pytest.mark.parametrize("is_signed", [False, True])
def test_key_range_matches_the_oracle(ds, n, is_signed):
    say(f"key range n={n} signed={is_signed}")
    rng = np.random.default_rng(n + 7 * is_signed)
    if n >= 1_000_000:
        g = torch.Generator(device="cuda")
        g.manual_seed(n)
        kd = torch.randint(-2**31, 2**31, (n,), generator=g, device=DEV, dtype=torch.int64).to(torch.int32)
        keys = w.as_u32(kd)
    else:
        keys = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        kd = torch.from_numpy(keys.view(np.int32).copy()).to(DEV)
    mm = torch.empty(2, dtype=torch.int32, device=DEV)
    ds.check(ds.dialsort_key_range(kd, mm, is_signed))
    torch.cuda.synchronize()
    got = tuple(int(v) for v in w.as_u32(mm))
    st, lo, hi = oracle.key_range(keys, is_signed)
    assert st == oracle.OK and got == (lo, hi)


def test_key_range_then_offset_sort(ds):
    """The min-max choice of phi: lo = min, U = max - min + 1, then the offset
    sort; signed keys in a narrow band far from zero."""
    rng = np.random.default_rng(11)
    keys = (rng.integers(-70_000, -10_000, 400_000)).astype(np.int32).view(np.uint32)
    kd = torch.from_numpy(keys.view(np.int32).copy()).to(DEV)
    mm = torch.empty(2, dtype=torch.int32, device=DEV)
    say("key range then offset sort")
    ds.check(ds.dialsort_key_range(kd, mm, True))
    lo, hi = (int(v) for v in mm.cpu())
    U = hi - lo + 1
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = torch.empty_like(kd)
    ws = ds.workspace(ds.dialsort_workspace_bytes(keys.size, U, ds.DIALSORT_MODE_SORT))
    ds.check(ds.dialsort_sort_offset(kd, lo, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    st, H_ref, out_ref = oracle.sort_offset(keys, lo, U)
    assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)
    assert np.array_equal(out.cpu().numpy(), np.sort(keys.view(np.int32)))
