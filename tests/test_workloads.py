"""The seeded input generators (no GPU)."""

from __future__ import annotations

import numpy as np
import torch

import workloads as w


def test_uniform_range_and_seed():
    a = w.as_u32(w.uniform(10_000, 366, 1))
    b = w.as_u32(w.uniform(10_000, 366, 1))
    assert np.array_equal(a, b) and a.max() < 366 and a.size == 10_000
    c = w.as_u32(w.uniform(1000, 1 << 32, 3))
    assert c.dtype == np.uint32 and c.max() > (1 << 31)  # the full 32-bit range is reachable


def test_zipf_rank_one_dominates():
    U, n, s = 1 << 16, 200_000, 1.2
    k = w.as_u32(w.zipf(n, U, s, 9))
    assert k.max() < U
    counts = np.bincount(k, minlength=U)
    cdf = w.zipf_table(U, s).numpy()
    p1 = cdf[0]
    top = counts.max() / n
    assert abs(top - p1) < 0.01  # the hottest key carries P(rank 1)


def test_hot_zipf_has_exact_hot_half():
    n, U = 100_000, 1 << 16
    k = w.as_u32(w.hot_zipf(n, U, 11))
    counts = np.bincount(k, minlength=U)
    assert counts.max() >= n // 2
    assert k.max() < U


def test_paper_skewed_mixture():
    n, U = 200_000, 256
    k = w.as_u32(w.paper_skewed(n, U, 2))
    small = (k <= (5 * U) // 100).mean()
    # 0.8 + 0.2 * (13/256)
    assert abs(small - (0.8 + 0.2 * 13 / 256)) < 0.01
    assert k.max() < U


def test_sorted_and_reverse():
    a = w.as_u32(w.paper_sorted(1000, 50, 3))
    b = w.as_u32(w.paper_reverse(1000, 50, 3))
    assert np.all(a[1:] >= a[:-1]) and np.all(b[1:] <= b[:-1])


def test_batch_spec():
    spec = w.batch_spec()
    assert len(spec) == 4096
    assert sum(s.dist == "zipf" for s in spec) == 2048
    ns = np.array([s.n for s in spec])
    Us = np.array([s.U for s in spec])
    assert ns.min() >= 1024 and ns.max() <= 4194304
    assert set(np.log2(Us).astype(int)) <= set(range(10, 21))
    assert w.batch_spec()[17].n == spec[17].n  # deterministic


def test_request_stream():
    r = w.request_stream(500, 200.0)
    t = np.array([x.arrival for x in r])
    assert np.all(np.diff(t) >= 0) and t[0] == 0.0
    assert {x.spec.U for x in r} <= {2**12, 2**16, 2**20, 2**24}
    assert all(4096 <= x.spec.n <= 2**24 for x in r)
    assert 150 < sum(x.spec.dist == "zipf" for x in r) < 350
