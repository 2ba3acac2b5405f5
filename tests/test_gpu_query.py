"""GPU parity of the queries on H (Sec. 3.3, the paragraph on the canonical
ordered state): frequency, presence, range-count, the running count P and
select, each compared element by element with the oracle on the same H.  H
comes from the oracle's own ingestion of seeded keys, so no input of these
tests comes from the GPU path."""

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


def dev_u64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(DEV)


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def run_queries(ds, H_np, keys_n, rng, nq=2000):
    U = H_np.size
    H = dev_u32(H_np)
    q = np.concatenate([rng.integers(0, U + 5, nq), [0, U - 1, U, 0xFFFFFFFF]]).astype(np.uint32)
    qd = dev_u32(q)
    out = torch.empty(q.size, dtype=torch.int32, device=DEV)
    ds.check(ds.dialsort_query_frequency(H, U, qd, out))
    assert np.array_equal(w.as_u32(out), oracle.frequency(H_np, q))
    pres = torch.empty(q.size, dtype=torch.uint8, device=DEV)
    ds.check(ds.dialsort_query_presence(H, U, qd, pres))
    assert np.array_equal(pres.cpu().numpy(), oracle.presence(H_np, q))
    # the running count, whole array
    P = torch.empty(U + 1, dtype=torch.int64, device=DEV)
    ws = ds.workspace(ds.dialsort_prefix_workspace_bytes(U))
    ds.check(ds.dialsort_prefix(H, U, P, ws))
    P_ref = oracle.prefix(H_np)
    P_np = host_u64(P)
    assert np.array_equal(P_np, P_ref)
    # range-count: ranges of every width, bounds past U, empty and reversed ranges
    a = rng.integers(0, U + 3, 300).astype(np.uint64)
    width = rng.integers(0, 1 + min(U, 5000), 300).astype(np.uint64)
    b = np.minimum(a + width, np.uint64(U + 3))
    a = np.concatenate([a, [0, 0, U, U + 9, 5, 2**40]]).astype(np.uint64)
    b = np.concatenate([b, [U, 2**40, U, U + 1, 2, 2**41]]).astype(np.uint64)
    rc = torch.empty(a.size, dtype=torch.int64, device=DEV)
    ds.check(ds.dialsort_query_range_count(P, U, dev_u64(a), dev_u64(b), rc))
    assert np.array_equal(host_u64(rc), oracle.range_count(H_np, a, b))
    # select: positions across the whole projection, and past its end
    r = np.concatenate([rng.integers(0, max(keys_n, 1), 200), [0, max(keys_n - 1, 0), keys_n, keys_n + 5]])
    r = r.astype(np.uint64)
    sel = torch.empty(r.size, dtype=torch.int32, device=DEV)
    ds.check(ds.dialsort_query_select(P, U, dev_u64(r), sel))
    assert np.array_equal(w.as_u32(sel), oracle.select(H_np, r))


@pytest.mark.parametrize("U,n", [(1, 10), (7, 1000), (300, 5000), (4096, 100000), (3 * 4096 + 17, 200000),
                                 (65536, 1 << 20), ((1 << 20) + 5, 3_000_000)])
def test_queries_match_the_oracle(ds, U, n):
    say(f"queries U={U} n={n}")
    rng = np.random.default_rng(U + n)
    keys = rng.integers(0, U, n).astype(np.uint32)
    st, H = oracle.histogram(keys, U)
    assert st == oracle.OK
    run_queries(ds, H, n, rng)


def test_queries_skewed_and_sparse(ds):
    rng = np.random.default_rng(5)
    U = 1 << 18
    say("queries on a Zipf(1.2) histogram and on a sparse one")
    keys = w.as_u32(w.zipf(2_000_000, U, 1.2, w.BASE_SEED + 31))
    st, H = oracle.histogram(keys, U)
    run_queries(ds, H, keys.size, rng)
    sparse = rng.choice(U, 40, replace=False).astype(np.uint32)
    st, H2 = oracle.histogram(sparse, U)
    run_queries(ds, H2, sparse.size, rng)
    empty = np.zeros(U, dtype=np.uint32)
    run_queries(ds, empty, 0, rng)


def test_prefix_at_the_large_workload_size(ds):
    U, n = 1 << 24, 10**8
    say("prefix and select at n = 1e8, U = 2^24")
    keys = w.as_u32(w.uniform(n, U, w.BASE_SEED + 1, "cuda"))
    st, H_np = oracle.histogram(keys, U)
    assert st == oracle.OK
    rng = np.random.default_rng(9)
    H = dev_u32(H_np)
    P = torch.empty(U + 1, dtype=torch.int64, device=DEV)
    ws = ds.workspace(ds.dialsort_prefix_workspace_bytes(U))
    ds.check(ds.dialsort_prefix(H, U, P, ws))
    assert np.array_equal(host_u64(P), oracle.prefix(H_np))
    # select at sampled positions, checked against the sorted keys
    r = np.sort(rng.integers(0, n, 64)).astype(np.uint64)
    sel = torch.empty(r.size, dtype=torch.int32, device=DEV)
    ds.check(ds.dialsort_query_select(P, U, dev_u64(r), sel))
    srt = np.sort(keys)
    assert np.array_equal(w.as_u32(sel), srt[r.astype(np.int64)])


def test_query_argument_errors(ds):
    U = 1000
    H = torch.zeros(U, dtype=torch.int32, device=DEV)
    q = torch.zeros(10, dtype=torch.int32, device=DEV)
    out = torch.zeros(10, dtype=torch.int32, device=DEV)
    assert ds.dialsort_query_frequency(H, 0, q, out) == ds.DIALSORT_EINVAL
    assert ds.dialsort_query_frequency(H, 2**32 + 1, q, out) == ds.DIALSORT_EINVAL
    assert ds.dialsort_query_frequency(H[1:], U - 1, q, out) == ds.DIALSORT_OK  # 4-byte aligned is enough
    bytes_ = torch.zeros(64, dtype=torch.uint8, device=DEV)
    mis = bytes_[1:41].view(torch.uint8)
    assert ds._lib.dialsort_query_frequency(ds._ptr(H), U, mis.data_ptr(), 10, ds._ptr(out), None) == \
        ds.DIALSORT_EINVAL
    P = torch.zeros(U + 1, dtype=torch.int64, device=DEV)
    small = torch.empty(8, dtype=torch.uint8, device=DEV)
    assert ds.dialsort_prefix(H, U, P, small) == ds.DIALSORT_EWORKSPACE
    assert ds.dialsort_prefix(H, U, P[:U], ds.workspace(ds.dialsort_prefix_workspace_bytes(U))) == \
        ds.DIALSORT_EINVAL
    # nothing to do: OK and nothing written
    empty = torch.empty(0, dtype=torch.int32, device=DEV)
    assert ds.dialsort_query_frequency(H, U, empty, empty) == ds.DIALSORT_OK
    torch.cuda.synchronize()
