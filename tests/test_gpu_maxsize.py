"""GPU checks at the largest input the library accepts, n = 2^32 - 1 keys
(counts and positions then use the whole 32-bit range), through properties
that hold at any size, computed on the device with plain torch ops:

  * partitioned sort, uniform keys, U = 2^24: H equals the keys' bincount,
    the output is nondecreasing with the same bincount, and sampled positions
    hold the key that the running count of H puts there (Eq. (2));
  * LDS-path sort of n equal keys, U = 2^16: one bin holds 2^32 - 1 and the
    output is that key everywhere;
  * DialSort-Radix over keys i * C mod 2^32 (C odd, so the keys are distinct
    and miss exactly one 32-bit value): the output is every value but that
    one, in unsigned and in signed order.
"""

from __future__ import annotations

import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
NMAX = (1 << 32) - 1
CHUNK = 1 << 30


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


@pytest.fixture(autouse=True)
def _free():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def chunks(n):
    for a in range(0, n, CHUNK):
        yield a, min(n, a + CHUNK)


def u32(t):
    return t.to(torch.int64) & 0xFFFFFFFF


def bincount(t, U):
    acc = torch.zeros(U, dtype=torch.int64, device=DEV)
    for a, b in chunks(t.numel()):
        acc += torch.bincount(t[a:b], minlength=U)
    return acc


def nondecreasing(t, signed):
    for a, b in chunks(t.numel()):
        lo = max(a - 1, 0)
        x = t[lo:b] if signed else u32(t[lo:b])
        if not bool((x[1:] >= x[:-1]).all()):
            return False
    return True


def test_partitioned_sort_at_max_n(ds):
    U = 1 << 24
    g = torch.Generator(device="cuda")
    g.manual_seed(20260321 + 77)
    keys = torch.randint(0, U, (NMAX,), generator=g, device=DEV, dtype=torch.int32)
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    out = torch.empty_like(keys)
    ws = ds.workspace(ds.dialsort_workspace_bytes(NMAX, U, ds.DIALSORT_MODE_SORT))
    say(f"partitioned sort n={NMAX} U={U}")
    ds.check(ds.dialsort_sort(keys, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    del ws
    Hl = u32(H)
    assert int(Hl.sum()) == NMAX
    assert torch.equal(bincount(keys, U), Hl)
    del keys
    assert nondecreasing(out, signed=True)  # keys < 2^24: int32 order is key order
    assert torch.equal(bincount(out, U), Hl)
    # sampled positions: out[r] is the k with P[k] <= r < P[k + 1]
    P = torch.cumsum(Hl, 0)  # P[k] = count of keys <= k
    r = torch.randint(0, NMAX, (1 << 16,), generator=g, device=DEV, dtype=torch.int64)
    r = torch.cat([r, torch.tensor([0, NMAX - 1], device=DEV)])
    k = torch.searchsorted(P, r, right=True)
    assert torch.equal(u32(out[r]), k)


def test_lds_sort_of_equal_keys_at_max_n(ds):
    U, key = 1 << 16, 12345
    keys = torch.full((NMAX,), key, dtype=torch.int32, device=DEV)
    H = torch.empty(U, dtype=torch.int32, device=DEV)
    ws = ds.workspace(ds.dialsort_workspace_bytes(NMAX, U, ds.DIALSORT_MODE_SORT))
    say(f"LDS-path sort of {NMAX} equal keys, in place")
    ds.check(ds.dialsort_sort(keys, U, H, keys, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    Hl = u32(H)
    assert int(Hl[key]) == NMAX and int(Hl.sum()) == NMAX
    for a, b in chunks(NMAX):
        assert bool((keys[a:b] == key).all())


@pytest.mark.parametrize("is_signed", [False, True])
def test_radix_at_max_n(ds, is_signed):
    C = 0x9E3779B1  # odd: i -> i * C mod 2^32 is a bijection of the 32-bit values
    keys = torch.empty(NMAX, dtype=torch.int32, device=DEV)
    for a, b in chunks(NMAX):
        i = torch.arange(a, b, dtype=torch.int64, device=DEV)
        v = (i * C) & 0xFFFFFFFF
        keys[a:b] = torch.where(v >= 1 << 31, v - (1 << 32), v).to(torch.int32)
        del i, v
    missing = (NMAX * C) & 0xFFFFFFFF  # the one value that index NMAX would have given
    out = torch.empty_like(keys)
    ws = ds.workspace(ds.dialsort_radix_workspace_bytes(NMAX))
    say(f"radix n={NMAX} signed={is_signed}")
    ds.check(ds.dialsort_sort_radix(keys, out, ws, is_signed=is_signed))
    torch.cuda.synchronize()
    del ws, keys
    # expected: every 32-bit value except `missing`, in the chosen order
    flip = (1 << 31) if is_signed else 0
    m = missing ^ flip  # rank of the missing value in that order
    for a, b in chunks(NMAX):
        i = torch.arange(a, b, dtype=torch.int64, device=DEV)
        want = ((i + (i >= m).to(torch.int64)) ^ flip) & 0xFFFFFFFF
        assert torch.equal(u32(out[a:b]), want), f"radix output differs in [{a}, {b})"
        del i, want
