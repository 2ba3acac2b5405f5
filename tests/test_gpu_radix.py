"""GPU parity of DialSort-Radix (LSD base 256, four passes) over the whole
32-bit range, unsigned and signed, against the oracle's radix sort (itself
pinned to numpy's sort)."""

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


def radix(ds, keys_u32, is_signed, in_place=False):
    n = keys_u32.size
    kd = torch.from_numpy(keys_u32.view(np.int32).copy()).to(DEV)
    out = kd if in_place else torch.empty(max(n, 1), dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_radix_workspace_bytes(n))
    ds.check(ds.dialsort_sort_radix(kd, out[:n], ws, is_signed=is_signed))
    torch.cuda.synchronize()
    return w.as_u32(out[:n])


@pytest.mark.parametrize("n", [0, 1, 2, 63, 65, 1023, 1025, 8191, 8192, 8193, 3 * 8192 + 5000, 100_000,
                               (1 << 20) + 3, 10_000_000])
@pytest.mark.parametrize("is_signed", [False, True])
def test_radix_random_full_range(ds, n, is_signed):
    say(f"radix n={n} signed={is_signed}")
    rng = np.random.default_rng(n * 2 + is_signed)
    keys = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    if n >= 4:
        keys[:4] = [0xFFFFFFFF, 0, 0x80000000, 0x7FFFFFFF]
    got = radix(ds, keys, is_signed)
    st, ref = oracle.sort_radix(keys, is_signed)
    assert st == oracle.OK
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("shape", ["sorted", "reverse", "equal", "one_digit", "few", "zipf"])
def test_radix_structured(ds, shape):
    n = 1_000_003
    rng = np.random.default_rng(7)
    base = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    if shape == "sorted":
        keys = np.sort(base)
    elif shape == "reverse":
        keys = np.sort(base)[::-1].copy()
    elif shape == "equal":
        keys = np.full(n, 0xDEADBEEF, dtype=np.uint32)
    elif shape == "one_digit":
        keys = (0x12003456 | (rng.integers(0, 256, n).astype(np.uint32) << 16)).astype(np.uint32)
    elif shape == "few":
        keys = rng.choice(np.array([5, 7, 0xFFFFFFFF, 1 << 31], dtype=np.uint32), n)
    else:
        keys = w.as_u32(w.zipf(n, 1 << 30, 1.2, w.BASE_SEED + 50)) * np.uint32(3)
    say(f"radix structured {shape}")
    for is_signed in (False, True):
        got = radix(ds, keys, is_signed)
        st, ref = oracle.sort_radix(keys, is_signed)
        assert np.array_equal(got, ref)


def test_radix_in_place_and_errors(ds):
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 2**32, 300_000, dtype=np.uint64).astype(np.uint32)
    say("radix in place")
    got = radix(ds, keys, True, in_place=True)
    assert np.array_equal(got.view(np.int32), np.sort(keys.view(np.int32)))
    kd = torch.zeros(100, dtype=torch.int32, device=DEV)
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    assert ds.dialsort_sort_radix(kd, kd, small) == ds.DIALSORT_EWORKSPACE
    ws = ds.workspace(ds.dialsort_radix_workspace_bytes(100))
    assert ds.dialsort_sort_radix(kd[:60], kd[40:100], ws) == ds.DIALSORT_EINVAL  # partial overlap
