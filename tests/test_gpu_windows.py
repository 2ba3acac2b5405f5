"""GPU parity of the tumbling-window sort, whose ingestion of one window
overlaps the projection of the previous one on a second stream (the streaming
remark of Sec. 4): every window's output and the last two histograms against
the oracle's sort of that window, the overlapped and the serial order give the
same bytes, and a key past U in one window is reported."""

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


def run_windows(ds, keys_u32, wn, count, U, two_streams=True):
    kd = torch.from_numpy(keys_u32.view(np.int32).copy()).to(DEV)
    H = torch.full((2 * U,), -1, dtype=torch.int32, device=DEV)
    out = torch.full((max(wn * count, 1),), -1, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_windows_workspace_bytes(wn, U))
    torch.cuda.synchronize()
    ingest = torch.cuda.Stream(device=DEV)
    project = torch.cuda.Stream(device=DEV) if two_streams else ingest
    ds.check(ds.dialsort_sort_windows(kd, wn, count, U, H, out[: wn * count], ws, ingest, project))
    st = ds.dialsort_status_sync(ws, project)
    torch.cuda.synchronize()
    return st, w.as_u32(H), w.as_u32(out[: wn * count])


@pytest.mark.parametrize("U,wn,count", [(1 << 16, 100_003, 5), (1000, 4097, 7), (1 << 20, 300_000, 4),
                                        (1 << 24, 2_000_000, 3), (1 << 12, 1, 3)])
def test_windows_match_the_oracle(ds, U, wn, count):
    say(f"windows U={U} window_n={wn} count={count}")
    rng = np.random.default_rng(U + wn + count)
    keys = rng.integers(0, U, wn * count).astype(np.uint32)
    if wn > 1000:
        keys[wn: wn + wn // 2] = 7  # a hot key in window 1
    st, H, out = run_windows(ds, keys, wn, count, U)
    assert st == ds.DIALSORT_OK
    for k in range(count):
        st_o, H_ref, out_ref = oracle.sort(keys[k * wn:(k + 1) * wn], U)
        assert st_o == oracle.OK
        assert np.array_equal(out[k * wn:(k + 1) * wn], out_ref), f"window {k}"
        if k >= count - 2:
            b = k % 2
            assert np.array_equal(H[b * U:(b + 1) * U], H_ref), f"histogram of window {k}"
    # the serial order (one stream) gives the same bytes
    st2, H2, out2 = run_windows(ds, keys, wn, count, U, two_streams=False)
    assert st2 == ds.DIALSORT_OK and np.array_equal(out2, out) and np.array_equal(H2, H)


def test_windows_report_a_key_past_U(ds):
    U, wn, count = 1 << 16, 50_000, 4
    rng = np.random.default_rng(3)
    keys = rng.integers(0, U, wn * count).astype(np.uint32)
    keys[2 * wn + 17] = U  # in window 2
    say("windows with a key past U")
    st, _, _ = run_windows(ds, keys, wn, count, U)
    assert st == ds.DIALSORT_ERANGE


def test_windows_argument_errors(ds):
    U, wn = 1 << 10, 1000
    kd = torch.zeros(3 * wn, dtype=torch.int32, device=DEV)
    H = torch.zeros(2 * U, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_windows_workspace_bytes(wn, U))
    assert ds.dialsort_sort_windows(kd, wn, 3, U, H, kd, ws) == ds.DIALSORT_EINVAL  # out == keys
    small = torch.empty(64, dtype=torch.uint8, device=DEV)
    out = torch.empty_like(kd)
    assert ds.dialsort_sort_windows(kd, wn, 3, U, H, out, small) == ds.DIALSORT_EWORKSPACE
    assert ds.dialsort_sort_windows(kd, wn, 3, U, H[:U], out, ws) == ds.DIALSORT_EINVAL  # H holds 2U


def test_back_to_back_calls_without_sync(ds):
    """Two calls on the same H and workspace, issued one after the other with
    no host synchronisation: the second call's first ingestions wait for the
    first call's last projections, so both calls' outputs are the oracle's."""
    U, wn, count = 1 << 16, 400_003, 3
    rng = np.random.default_rng(29)
    k1 = rng.integers(0, U, wn * count).astype(np.uint32)
    k2 = rng.integers(0, U, wn * count).astype(np.uint32)
    k2[:wn // 2] = 5  # a hot key in the second call's first window
    d1 = torch.from_numpy(k1.view(np.int32).copy()).to(DEV)
    d2 = torch.from_numpy(k2.view(np.int32).copy()).to(DEV)
    H = torch.full((2 * U,), -1, dtype=torch.int32, device=DEV)
    o1 = torch.full((wn * count,), -1, dtype=torch.int32, device=DEV)
    o2 = torch.full((wn * count,), -1, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_windows_workspace_bytes(wn, U))
    torch.cuda.synchronize()
    ingest = torch.cuda.Stream(device=DEV)
    project = torch.cuda.Stream(device=DEV)
    say(f"two window calls back to back U={U} window_n={wn} count={count}")
    ds.check(ds.dialsort_sort_windows(d1, wn, count, U, H, o1, ws, ingest, project))
    ds.check(ds.dialsort_sort_windows(d2, wn, count, U, H, o2, ws, ingest, project))
    assert ds.dialsort_status_sync(ws, project) == ds.DIALSORT_OK
    torch.cuda.synchronize()
    out1, out2, Hh = w.as_u32(o1), w.as_u32(o2), w.as_u32(H)
    for keys, out in ((k1, out1), (k2, out2)):
        for k in range(count):
            st_o, _, out_ref = oracle.sort(keys[k * wn:(k + 1) * wn], U)
            assert st_o == oracle.OK
            assert np.array_equal(out[k * wn:(k + 1) * wn], out_ref), f"window {k}"
    for k in (count - 2, count - 1):
        _, H_ref, _ = oracle.sort(k2[k * wn:(k + 1) * wn], U)
        b = k % 2
        assert np.array_equal(Hh[b * U:(b + 1) * U], H_ref), f"histogram of window {k}"
