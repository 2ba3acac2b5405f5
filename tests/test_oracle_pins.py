"""Pins for the CPU oracle (no GPU).

The oracle states Eq. (1) and Eq. (2) of DialSort Sec. 3.3.  These tests tie it
to things other than itself:
  * the paper's worked examples (tests/golden, each file cites its figure);
  * brute force on every sequence over U <= 3 of length <= 7 (count by equality,
    order by a comparison sort -- the textbook definition of a sorted multiset);
  * numpy's bincount and sort on random inputs (library routines that reduce to
    the same definition);
  * Theorem "thm:correct": nondecreasing output, multiset equality, sum H = n;
  * the error readings (key >= U, U out of range, out_cap below sum H).
A last group plants plausible mistakes in copies of the oracle's two steps and
checks that these pins reject every one of them.
"""

from __future__ import annotations

import ctypes
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            d[k] = v
    return d


def ints(s):
    return [int(x) for x in s.split()]


# --- worked examples --------------------------------------------------------

def test_fig_viz_ingestion_and_projection():
    g = read_golden("fig_viz.txt")
    st, H, out = oracle.sort(ints(g["keys"]), int(g["U"]))
    assert st == oracle.OK
    assert H.tolist() == ints(g["H"])
    assert out.tolist() == ints(g["out"])


def test_fig_viz_in_place():
    g = read_golden("fig_viz.txt")
    st, H, out = oracle.sort(ints(g["keys"]), int(g["U"]), in_place=True)
    assert st == oracle.OK and out.tolist() == ints(g["out"])


@pytest.mark.parametrize("name", ["fig_abacus.txt", "fig_physical.txt", "fig_viz.txt"])
def test_projection_examples(name):
    g = read_golden(name)
    st, out = oracle.reconstruct(ints(g["H"]))
    assert st == oracle.OK
    assert out.tolist() == ints(g["out"])
    # and ingestion of that output gives back H
    st, H = oracle.histogram(out, int(g["U"]))
    assert st == oracle.OK and H.tolist() == ints(g["H"])


# --- exhaustive brute force -------------------------------------------------

def brute_hist(seq, U):
    return [sum(1 for x in seq if x == k) for k in range(U)]


def test_exhaustive_small_universes():
    cases = 0
    for U in (1, 2, 3):
        for length in range(0, 8):
            for seq in itertools.product(range(U), repeat=length):
                st, H, out = oracle.sort(list(seq), U)
                assert st == oracle.OK
                assert H.tolist() == brute_hist(seq, U)
                assert out.tolist() == sorted(seq)
                cases += 1
    assert cases == sum(U ** L for U in (1, 2, 3) for L in range(8))


# --- library routines and Theorem "thm:correct" ------------------------------

@pytest.mark.parametrize("U", [1, 2, 6, 128, 255, 256, 366, 1000, 1024, 4097, 65536, 65537, 1 << 20])
@pytest.mark.parametrize("n", [0, 1, 7, 1000, 100_003])
def test_against_numpy(U, n):
    rng = np.random.default_rng(U * 7919 + n)
    keys = rng.integers(0, U, n, dtype=np.uint64).astype(np.uint32)
    st, H, out = oracle.sort(keys, U)
    assert st == oracle.OK
    assert np.array_equal(H, np.bincount(keys, minlength=U).astype(np.uint32))
    assert np.array_equal(out, np.sort(keys))
    # Theorem "thm:correct": nondecreasing, multiset-equal, length n
    assert int(H.sum(dtype=np.uint64)) == n and out.size == n
    assert np.all(out[1:] >= out[:-1])
    assert np.array_equal(np.bincount(out, minlength=U).astype(np.uint32), H)


def test_paper_distributions():
    import workloads

    for name, gen in workloads.PAPER_DISTRIBUTIONS.items():
        for U in (256, 1024, 65536):
            keys = workloads.as_u32(gen(20_000, U, workloads.BASE_SEED))
            st, H, out = oracle.sort(keys, U)
            assert st == oracle.OK, name
            assert np.array_equal(out, np.sort(keys)), name
            assert np.array_equal(H, np.bincount(keys, minlength=U).astype(np.uint32)), name


def test_keys_near_top_of_universe():
    U = (1 << 31) + 5
    # only the top of the universe is touched; H is allocated in full, so keep U modest
    U = (1 << 26) + 3
    keys = np.array([U - 1, 0, U - 1, U - 2, 5], dtype=np.uint32)
    st, H, out = oracle.sort(keys, U)
    assert st == oracle.OK
    assert out.tolist() == sorted(keys.tolist())
    assert H[U - 1] == 2 and H[U - 2] == 1 and H[0] == 1 and H[5] == 1


# --- errors ---------------------------------------------------------------

def test_key_out_of_range():
    st, H = oracle.histogram([0, 1, 6], 6)
    assert st == oracle.ERANGE
    st, H, out = oracle.sort([7], 7)
    assert st == oracle.ERANGE


def test_bad_universe():
    lib = oracle._load()
    H = np.zeros(4, dtype=np.uint32)
    assert lib.oracle_histogram(None, 0, 0, H.ctypes.data_as(ctypes.c_void_p)) == oracle.EINVAL
    assert lib.oracle_histogram(None, 0, (1 << 32) + 1, H.ctypes.data_as(ctypes.c_void_p)) == oracle.EINVAL


def test_count_overflow_guard():
    lib = oracle._load()
    H = np.zeros(4, dtype=np.uint32)
    k = np.zeros(1, dtype=np.uint32)
    # rejected before any key is read
    assert lib.oracle_histogram(k.ctypes.data_as(ctypes.c_void_p), 1 << 32, 4,
                                H.ctypes.data_as(ctypes.c_void_p)) == oracle.EOVERFLOW


def test_reconstruct_capacity():
    st, out = oracle.reconstruct([1, 2, 0, 3, 1, 2], 4)
    assert st == oracle.EOVERFLOW and out.tolist() == [0, 1, 1, 3]
    st, out = oracle.reconstruct([1, 2, 0, 3, 1, 2], 100)
    assert st == oracle.OK and out.tolist() == [0, 1, 1, 3, 3, 3, 4, 5, 5]
    st, out = oracle.reconstruct([0, 0, 0], 0)
    assert st == oracle.OK and out.size == 0
    st, out = oracle.reconstruct([0, 0, 0], 5)  # nothing to emit, room to spare
    assert st == oracle.OK and out.size == 0


# --- planted mistakes: every one must be rejected by the pins above ----------

def pins_accept(hist_fn, proj_fn) -> bool:
    """True if a (histogram, projection) pair passes the worked examples, the
    exhaustive check and a numpy comparison."""
    for name in ("fig_viz.txt",):
        g = read_golden(name)
        H = hist_fn(ints(g["keys"]), int(g["U"]))
        if list(H) != ints(g["H"]) or list(proj_fn(H)) != ints(g["out"]):
            return False
    for name in ("fig_abacus.txt", "fig_physical.txt"):
        g = read_golden(name)
        if list(proj_fn(ints(g["H"]))) != ints(g["out"]):
            return False
    for U in (1, 2, 3):
        for length in range(0, 6):
            for seq in itertools.product(range(U), repeat=length):
                H = hist_fn(list(seq), U)
                if list(H) != brute_hist(seq, U) or list(proj_fn(H)) != sorted(seq):
                    return False
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 300, 5000)
    H = hist_fn(keys.tolist(), 300)
    return list(H) == np.bincount(keys, minlength=300).tolist() and list(proj_fn(H)) == sorted(keys.tolist())


def good_hist(keys, U):
    H = [0] * U
    for x in keys:
        H[x] += 1
    return H


def good_proj(H):
    out = []
    for k, c in enumerate(H):
        out.extend([k] * c)
    return out


def test_pins_accept_the_plain_definition():
    assert pins_accept(good_hist, good_proj)


MUTANTS = {
    "drops the last key": (lambda keys, U: good_hist(keys[:-1], U), good_proj),
    "counts key x into x-1": (lambda keys, U: good_hist([max(x - 1, 0) for x in keys], U), good_proj),
    "descending projection": (good_hist, lambda H: good_proj(H)[::-1]),
    "emits each present key once": (good_hist, lambda H: [k for k, c in enumerate(H) if c]),
    "skips bin 0": (good_hist, lambda H: good_proj([0] + list(H[1:]))),
    "off-by-one emission count": (good_hist, lambda H: good_proj([c + 1 if c else 0 for c in H])),
    "stops one bin early": (good_hist, lambda H: good_proj(list(H[:-1]))),
    "emits k+1": (good_hist, lambda H: [x + 1 for x in good_proj(H)]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistakes(name):
    h, p = MUTANTS[name]
    assert not pins_accept(h, p), name


# ---- queries on H (Sec. 3.3, the paragraph on the canonical ordered state) ----
# Each is pinned to the keys themselves (not to H): counting, membership and
# order statistics of the input multiset computed by numpy.


@pytest.mark.parametrize("U,n", [(1, 5), (7, 40), (300, 1000), (4096, 20000), (70000, 5000)])
def test_queries_against_the_keys(U, n):
    rng = np.random.default_rng(U * 31 + n)
    keys = rng.integers(0, U, n).astype(np.uint32)
    st, H = oracle.histogram(keys, U)
    assert st == oracle.OK
    q = np.concatenate([rng.integers(0, U + 3, 200), [0, U - 1, U, 0xFFFFFFFF]]).astype(np.uint32)
    # frequency(k): how many keys equal k, by comparing every key with k
    freq = np.array([np.count_nonzero(keys == x) for x in q], dtype=np.uint32)
    assert np.array_equal(oracle.frequency(H, q), freq)
    # presence(k): does k occur among the keys
    assert np.array_equal(oracle.presence(H, q), np.isin(q, keys).astype(np.uint8))
    # range-count(a, b): keys with a <= x < b, bounds beyond U included
    a = rng.integers(0, U + 5, 100).astype(np.uint64)
    b = rng.integers(0, U + 5, 100).astype(np.uint64)
    a = np.concatenate([a, [0, 0, U, 2**33]]).astype(np.uint64)
    b = np.concatenate([b, [U, 2**33, U, 2**34]]).astype(np.uint64)
    k64 = keys.astype(np.uint64)
    want = np.array([np.count_nonzero((k64 >= x) & (k64 < y)) for x, y in zip(a, b)], dtype=np.uint64)
    assert np.array_equal(oracle.range_count(H, a, b), want)
    # prefix: P[k] = number of keys below k
    P = oracle.prefix(H)
    assert P.size == U + 1 and P[0] == 0 and P[U] == n
    ks = np.unique(np.concatenate([rng.integers(0, U + 1, 50), [0, U]]))
    assert np.array_equal(P[ks], np.array([np.count_nonzero(k64 < x) for x in ks], dtype=np.uint64))
    # select(r): the r-th smallest key (np.sort, a comparison sort), past the end 0xFFFFFFFF
    r = np.concatenate([rng.integers(0, n, 100), [0, n - 1, n, n + 7]]).astype(np.uint64)
    srt = np.sort(keys)
    want_sel = np.array([srt[int(x)] if x < n else 0xFFFFFFFF for x in r], dtype=np.uint32)
    assert np.array_equal(oracle.select(H, r), want_sel)


def test_queries_on_the_worked_example():
    # the abacus example's histogram (Fig. fig:abacus caption): H = [1,2,0,3,1,2]
    H = np.array([1, 2, 0, 3, 1, 2], dtype=np.uint32)
    assert list(oracle.frequency(H, [0, 1, 2, 3, 6])) == [1, 2, 0, 3, 0]
    assert list(oracle.presence(H, [2, 3, 5, 6])) == [0, 1, 1, 0]
    assert list(oracle.range_count(H, [0, 1, 3, 4], [6, 4, 4, 2])) == [9, 5, 3, 0]
    assert list(oracle.prefix(H)) == [0, 1, 3, 3, 6, 7, 9]
    # the projection <0,1,1,3,3,3,4,5,5>, read position by position
    assert list(oracle.select(H, range(10))) == [0, 1, 1, 3, 3, 3, 4, 5, 5, 0xFFFFFFFF]


def test_accumulate_is_ingestion_of_the_whole_stream():
    """Ingesting a stream piece by piece gives the histogram of the whole stream
    (numpy's bincount of the concatenation); a count past 2^32 - 1 overflows."""
    rng = np.random.default_rng(77)
    U = 5000
    pieces = [rng.integers(0, U, m).astype(np.uint32) for m in (0, 1, 999, 4096, 17, 20000)]
    H = np.zeros(U, dtype=np.uint32)
    for p in pieces:
        st, H = oracle.histogram_accumulate(p, U, H)
        assert st == oracle.OK
    whole = np.concatenate(pieces)
    assert np.array_equal(H, np.bincount(whole, minlength=U).astype(np.uint32))
    st, H2 = oracle.histogram_accumulate(np.array([U], dtype=np.uint32), U, H)
    assert st == oracle.ERANGE
    near = np.zeros(4, dtype=np.uint32)
    near[2] = 0xFFFFFFFE
    st, near = oracle.histogram_accumulate(np.array([2], dtype=np.uint32), 4, near)
    assert st == oracle.OK and near[2] == 0xFFFFFFFF
    st, _ = oracle.histogram_accumulate(np.array([2], dtype=np.uint32), 4, near)
    assert st == oracle.EOVERFLOW


def test_offset_sort_is_the_order_of_the_domain():
    """phi(x) = x - lo (Sec. 3.4): signed int32 keys come out in numpy's signed
    order, and a universe that wraps past 2^32 - 1 keeps its order."""
    rng = np.random.default_rng(91)
    signed = rng.integers(-1000, 1001, 5000).astype(np.int32)
    lo = -1000
    st, H, out = oracle.sort_offset(signed.view(np.uint32), lo, 2001)
    assert st == oracle.OK
    assert np.array_equal(out.view(np.int32), np.sort(signed))
    assert H[0] == np.count_nonzero(signed == -1000) and H[2000] == np.count_nonzero(signed == 1000)
    lo = 0xFFFFFF00
    wrap = ((lo + rng.integers(0, 512, 3000)) % 2**32).astype(np.uint32)
    st, H, out = oracle.sort_offset(wrap, lo, 512)
    assert st == oracle.OK
    want = sorted(wrap.tolist(), key=lambda x: (x - lo) % 2**32)
    assert out.tolist() == want
    st, _, _ = oracle.sort_offset(np.array([lo - 1], dtype=np.uint32), lo, 512)
    assert st == oracle.ERANGE
    st, H0, out0 = oracle.sort_offset(signed.view(np.uint32) & 0, 0, 1)  # lo = 0 is the plain sort
    assert st == oracle.OK and H0[0] == signed.size


@pytest.mark.parametrize("n", [0, 1, 2, 255, 1000, 70000])
def test_radix_is_numpy_sort(n):
    """DialSort-Radix over the full 32-bit range, signed and unsigned, equals a
    comparison sort (numpy) -- including keys that differ only in one digit."""
    rng = np.random.default_rng(n + 3)
    u = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    if n >= 4:
        u[:4] = [0xFFFFFFFF, 0, 0x80000000, 0x7FFFFFFF]
    st, out = oracle.sort_radix(u)
    assert st == oracle.OK and np.array_equal(out, np.sort(u))
    s = u.view(np.int32)
    st, out = oracle.sort_radix(s, is_signed=True)
    assert st == oracle.OK and np.array_equal(out.view(np.int32), np.sort(s))
    # one digit at a time: keys equal above and below digit 2
    d = (0x11220033 | (rng.integers(0, 256, n).astype(np.uint32) << 8)).astype(np.uint32)
    st, out = oracle.sort_radix(d)
    assert np.array_equal(out, np.sort(d))


def test_lut_sort_orders_a_non_integer_domain():
    """phi^-1 as a table (Sec. 3.4): weekday names indexed by their position in
    the week come out in week order, whatever order the input holds them in;
    with an increasing table the output is the comparison sort of the decoded
    values; with any table it is the table read at the sorted indices."""
    week = ["Mon", "Tue", "Wed", "Thu", "Fri", "Sat", "Sun"]
    codes = {name: i for i, name in enumerate(week)}
    rng = np.random.default_rng(17)
    days = [week[i] for i in rng.integers(0, 7, 200)]
    # the table decodes an index into a token of the name (its bytes as an int)
    token = np.array([int.from_bytes(d.encode(), "little") for d in week], dtype=np.uint32)
    name_of = {int(t): d for t, d in zip(token, week)}
    keys = np.array([codes[d] for d in days], dtype=np.uint32)
    st, H, out = oracle.sort_lut(keys, 7, token)
    assert st == oracle.OK
    assert [name_of[int(t)] for t in out] == sorted(days, key=week.index)
    assert H.tolist() == [days.count(d) for d in week]
    # an increasing table: the order of the decoded values themselves
    U = 5000
    inc = np.cumsum(rng.integers(1, 1000, U)).astype(np.uint32)
    idx = rng.integers(0, U, 20000).astype(np.uint32)
    st, _, out = oracle.sort_lut(idx, U, inc)
    assert st == oracle.OK and np.array_equal(out, np.sort(inc[idx]))
    # any table (here a permutation): the table at the sorted indices
    perm = rng.permutation(U).astype(np.uint32)
    st, _, out = oracle.sort_lut(idx, U, perm)
    assert st == oracle.OK and np.array_equal(out, perm[np.sort(idx)])
    st, _, _ = oracle.sort_lut(np.array([U], dtype=np.uint32), U, perm)
    assert st == oracle.ERANGE
    st, _, out = oracle.sort_lut(np.array([], dtype=np.uint32), U, perm)
    assert st == oracle.OK and out.size == 0


@pytest.mark.parametrize("n", [0, 1, 2, 1000, 100_003])
def test_key_range_is_numpy_min_max(n):
    """The key range that fixes the smallest offset map (Sec. 3.4), unsigned
    and signed, against numpy's min and max; the empty input leaves min above
    max."""
    rng = np.random.default_rng(n + 29)
    u = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    st, lo, hi = oracle.key_range(u)
    assert st == oracle.OK
    if n:
        assert (lo, hi) == (int(u.min()), int(u.max()))
        s = u.view(np.int32)
        st, lo, hi = oracle.key_range(u, is_signed=True)
        assert (np.uint32(lo).view(np.int32), np.uint32(hi).view(np.int32)) == (s.min(), s.max())
    else:
        assert (lo, hi) == (0xFFFFFFFF, 0)
        assert oracle.key_range(u, is_signed=True)[1:] == (0x7FFFFFFF, 0x80000000)
    # the extremes themselves
    ext = np.array([0x80000000, 0x7FFFFFFF, 0, 0xFFFFFFFF], dtype=np.uint32)
    assert oracle.key_range(ext)[1:] == (0, 0xFFFFFFFF)
    assert oracle.key_range(ext, is_signed=True)[1:] == (0x80000000, 0x7FFFFFFF)
