"""The later entry points on inputs that start at an odd 4-byte offset (not
16-byte aligned) and on ragged sizes, against the oracle: DialSort-Radix, the
lookup-table sort, the key range and the windowed sort."""

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


def at_offset(arr_u32, off):
    """A device copy of arr whose first element sits `off` words into its buffer."""
    buf = torch.zeros(arr_u32.size + off + 4, dtype=torch.int32, device=DEV)
    t = buf[off:off + arr_u32.size]
    t.copy_(torch.from_numpy(arr_u32.view(np.int32).copy()))
    return t


@pytest.mark.parametrize("off", [1, 2, 3])
def test_radix_unaligned(ds, off):
    n = 123_457
    keys = np.random.default_rng(off).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    kd = at_offset(keys, off)
    out = at_offset(np.zeros(n, dtype=np.uint32), 4 - off)
    ws = ds.workspace(ds.dialsort_radix_workspace_bytes(n))
    say(f"radix unaligned off={off}")
    ds.check(ds.dialsort_sort_radix(kd, out, ws, is_signed=True))
    torch.cuda.synchronize()
    st, ref = oracle.sort_radix(keys, True)
    assert np.array_equal(w.as_u32(out), ref)


@pytest.mark.parametrize("off", [1, 3])
def test_lut_sort_and_key_range_unaligned(ds, off):
    U, n = 5000, 77_777
    rng = np.random.default_rng(10 + off)
    keys = rng.integers(0, U, n).astype(np.uint32)
    lut = np.cumsum(rng.integers(1, 9, U)).astype(np.uint32)
    kd, lutd = at_offset(keys, off), at_offset(lut, off)
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = at_offset(np.zeros(n, dtype=np.uint32), 2)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT))
    say(f"lut sort unaligned off={off}")
    ds.check(ds.dialsort_sort_lut(kd, U, lutd, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    st, H_ref, out_ref = oracle.sort_lut(keys, U, lut)
    assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)
    mm = torch.empty(2, dtype=torch.int32, device=DEV)
    ds.check(ds.dialsort_key_range(kd, mm, False))
    torch.cuda.synchronize()
    assert tuple(int(v) for v in w.as_u32(mm)) == oracle.key_range(keys)[1:]


def test_windows_unaligned(ds):
    U, wn, count = 1 << 16, 33_333, 3
    keys = np.random.default_rng(4).integers(0, U, wn * count).astype(np.uint32)
    kd = at_offset(keys, 1)
    out = at_offset(np.zeros(wn * count, dtype=np.uint32), 3)
    H = torch.empty(2 * U, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_windows_workspace_bytes(wn, U))
    say("windows unaligned")
    ds.check(ds.dialsort_sort_windows(kd, wn, count, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    got = w.as_u32(out)
    for k in range(count):
        assert np.array_equal(got[k * wn:(k + 1) * wn], oracle.sort(keys[k * wn:(k + 1) * wn], U)[2])
