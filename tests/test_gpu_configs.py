"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (one dialsort_sort / dialsort_histogram call,
inputs resident on the device).  Every case is compared with the oracle on the
whole output, bit-exactly.

  plain:   n = 2^20 uniform keys, U = 2^16 (seeds 20260321 + 0..4)
  large:   n = 10^8 uniform keys, U = 2^24, sort and histogram-only
  skewed:  n = 2^28, U = 2^16, half the keys one hot value, the rest Zipf(1.2)
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


def check_sort(ds, keys_dev, U, label):
    n = keys_dev.numel()
    dev = keys_dev.device
    H = torch.empty(U, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT), dev)
    say(f"{label} sort n={n} U={U}")
    ds.check(ds.dialsort_sort(keys_dev, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    kh = w.as_u32(keys_dev)
    st, H_ref, out_ref = oracle.sort(kh, U)
    assert st == oracle.OK
    assert np.array_equal(w.as_u32(H), H_ref), f"{label}: H differs"
    oh = w.as_u32(out)
    del out
    assert np.array_equal(oh, out_ref), f"{label}: output differs"
    return H_ref


@pytest.mark.parametrize("s", range(5))
def test_plain_2pow20(ds, s):
    keys = w.uniform(1 << 20, 1 << 16, w.BASE_SEED + s, "cuda")
    check_sort(ds, keys, 1 << 16, f"plain seed+{s}")


def test_large_uniform_1e8(ds):
    U = 1 << 24
    keys = w.uniform(10**8, U, w.BASE_SEED + 1, "cuda")
    H_ref = check_sort(ds, keys, U, "large")
    H = torch.empty(U, dtype=torch.int32, device=keys.device)
    ws = ds.workspace(ds.dialsort_workspace_bytes(keys.numel(), U, ds.DIALSORT_MODE_HISTOGRAM), keys.device)
    say("large histogram-only")
    ds.check(ds.dialsort_histogram(keys, U, H, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    assert np.array_equal(w.as_u32(H), H_ref)


def test_skewed_2pow28(ds):
    U = 1 << 16
    keys = w.hot_zipf(1 << 28, U, w.BASE_SEED + 2, "cuda")
    H_ref = check_sort(ds, keys, U, "skewed")
    assert H_ref.max() >= (1 << 27)


def test_many_heavy_buckets(ds):
    """U = 2^20 (16 buckets of 2^16 bins) with 70e6 uniform keys: every bucket
    holds more than 2^22 keys, so each is counted and projected in two halves --
    32 spans of fill items, which must all fit the item list."""
    keys = w.uniform(70_000_000, 1 << 20, w.BASE_SEED + 9, "cuda")
    check_sort(ds, keys, 1 << 20, "heavy buckets")


def check_hist(ds, keys_dev, U, H_ref, label):
    H = torch.empty(U, dtype=torch.int32, device=keys_dev.device)
    ws = ds.workspace(ds.dialsort_workspace_bytes(keys_dev.numel(), U, ds.DIALSORT_MODE_HISTOGRAM), keys_dev.device)
    say(f"{label} histogram-only n={keys_dev.numel()} U={U}")
    ds.check(ds.dialsort_histogram(keys_dev, U, H, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    assert np.array_equal(w.as_u32(H), H_ref), f"{label}: histogram-only H differs"


def test_split_zipf_large_universe(ds):
    """Zipf(1.2) keys over a random permutation of [0, 2^24): the buckets of the
    most frequent keys hold millions of keys each and are counted by several
    workgroups that add into H; the last of them projects the bucket."""
    U = 1 << 24
    keys = w.zipf(1 << 24, U, 1.2, w.BASE_SEED + 21, "cuda")
    H_ref = check_sort(ds, keys, U, "split zipf")
    per_bucket = H_ref.reshape(-1, 1 << 16).sum(axis=1, dtype=np.int64)
    assert per_bucket.max() > 2 * (1 << 18)  # at least one bucket is split
    check_hist(ds, keys, U, H_ref, "split zipf")


def test_split_hot_key_wraps_packed_fields(ds):
    """Half of 2^22 keys are one value: each part of its bucket sees far more
    than 0xFFFF of it, so the part recounts its bins in two 32-bit halves."""
    U = 1 << 20
    keys = w.hot_zipf(1 << 22, U, w.BASE_SEED + 22, "cuda")
    H_ref = check_sort(ds, keys, U, "split hot key")
    assert H_ref.max() >= (1 << 21)
    check_hist(ds, keys, U, H_ref, "split hot key")


def test_split_one_bucket_every_bin(ds):
    """2^23 keys uniform over the 2^16 bins of bucket 5 of U = 2^20: 32 parts
    each add a nonzero count to nearly every bin of the bucket."""
    U = 1 << 20
    keys = w.uniform(1 << 23, 1 << 16, w.BASE_SEED + 23, "cuda") + (5 << 16)
    H_ref = check_sort(ds, keys, U, "split one bucket")
    assert H_ref[5 << 16:6 << 16].min() > 0
    check_hist(ds, keys, U, H_ref, "split one bucket")
