"""The allocation-free sort (dialsort_sort_noalloc) against dialsort_sort
through the C ABI: two calls in a row on the library's shared per-device
workspace, the second with a smaller input, must give exactly dialsort_sort's
H and output; the status word reports a key past U; a sort whose workspace
would exceed the library's array is refused before anything runs."""

from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


def with_workspace(ds, keys, U):
    n = keys.numel()
    H = torch.full((U,), -1, dtype=torch.int32, device=DEV)
    out = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT))
    ds.check(ds.dialsort_sort(keys, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    return H, out


def test_noalloc_equals_sort_on_two_calls(ds):
    cases = [(3_000_017, 1 << 23, "uniform"), (100_003, 1 << 16, "zipf")]
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    results = []
    for i, (n, U, dist) in enumerate(cases):
        spec = w.ArraySpec(n, U, dist, 1.2, w.BASE_SEED + 600 + i)
        keys = spec.keys("cpu").to(DEV)
        H = torch.full((U,), -1, dtype=torch.int32, device=DEV)
        out = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        say(f"noalloc call {i}: n={n} U={U} {dist}")
        ds.check(ds.dialsort_sort_noalloc(keys, U, H, out, status))
        results.append((keys, U, H, out))
    # both calls were enqueued back to back; compare after both ran
    torch.cuda.synchronize()
    assert int(status[0]) == 0
    for keys, U, H, out in results:
        H_ref, out_ref = with_workspace(ds, keys, U)
        assert torch.equal(H, H_ref)
        assert torch.equal(out, out_ref)


def test_noalloc_status_and_limits(ds):
    U = 1 << 20
    keys = w.uniform(50_000, U, w.BASE_SEED + 610).to(DEV)
    keys[4321] = U
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = torch.empty(keys.numel(), dtype=torch.int32, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    say("noalloc key past U")
    ds.check(ds.dialsort_sort_noalloc(keys, U, H, out, status))
    torch.cuda.synchronize()
    assert int(status[0]) & 1
    # the next call on the shared workspace starts clean
    keys[4321] = 5
    say("noalloc clean call after an error")
    ds.check(ds.dialsort_sort_noalloc(keys, U, H, out, status))
    torch.cuda.synchronize()
    assert int(status[0]) == 0
    H_ref, out_ref = with_workspace(ds, keys, U)
    assert torch.equal(H, H_ref) and torch.equal(out, out_ref)
    # a workspace beyond the library's array: refused before any launch
    big_n = 200_000_000
    assert ds.dialsort_workspace_bytes(big_n, 1 << 24, ds.DIALSORT_MODE_SORT) > (64 << 20)
    kb = torch.empty(big_n, dtype=torch.int32, device=DEV)
    Hb = torch.empty(1 << 24, dtype=torch.int32, device=DEV)
    assert ds.dialsort_sort_noalloc(kb, 1 << 24, Hb, kb, None) == ds.DIALSORT_EWORKSPACE
