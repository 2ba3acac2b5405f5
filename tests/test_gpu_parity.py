"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Every case prints its name before touching the GPU.  Sizes span several tiles
and ragged tails for every ingestion path:
  LDS32 (U <= 32768), LDS16 packed (32768 < U <= 65536), the U-partitioned path
  (65536 < U <= 2^28) and direct global atomics (tiny n next to U, or U > 2^28),
plus the look-back scan and the chunked fill.  Integer work, so the bar is exact
equality of H and of the sorted output.
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

SEED = w.BASE_SEED


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


def gpu_sort(ds, keys, U, mode="sort", in_place=False):
    n = keys.numel()
    H = torch.full((U,), -1, dtype=torch.int32, device=keys.device)  # garbage: must be overwritten
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT if mode == "sort"
                                                  else ds.DIALSORT_MODE_HISTOGRAM), keys.device)
    if mode == "sort":
        out = keys if in_place else torch.full((n,), -7, dtype=torch.int32, device=keys.device)
        ds.check(ds.dialsort_sort(keys, U, H, out, ws))
    else:
        out = None
        ds.check(ds.dialsort_histogram(keys, U, H, ws))
    st = ds.dialsort_status_sync(ws)
    return st, H, out


def assert_parity(ds, keys_host, U, keys_dev=None, mode="sort", in_place=False, label=""):
    dev = torch.device("cuda:0")
    if keys_dev is None:
        keys_dev = torch.from_numpy(keys_host.view(np.int32)).to(dev)
    say(f"{label} n={keys_host.size} U={U} mode={mode} in_place={in_place}")
    st, H, out = gpu_sort(ds, keys_dev, U, mode, in_place)
    assert st == ds.DIALSORT_OK, ds.dialsort_strerror(st)
    ost, H_ref, out_ref = oracle.sort(keys_host, U)
    assert ost == oracle.OK
    Hh = w.as_u32(H)
    if not np.array_equal(Hh, H_ref):
        bad = np.nonzero(Hh != H_ref)[0]
        raise AssertionError(f"H differs at {bad.size} bins, first {bad[:5]}: {Hh[bad[:5]]} vs {H_ref[bad[:5]]}")
    if mode == "sort":
        oh = w.as_u32(out)
        if not np.array_equal(oh, out_ref):
            bad = np.nonzero(oh != out_ref)[0]
            raise AssertionError(f"out differs at {bad.size} positions, first {bad[:5]}")


UNIVERSES = [1, 2, 6, 128, 366, 1000, 4096, 4097, 32768, 32769, 40001, 65535, 65536, 65537, 1 << 17,
             (1 << 20) + 1, (1 << 24) + 3]
SIZES = [0, 1, 5, 1000, 65539, (1 << 20) + 7]


@pytest.mark.parametrize("U", UNIVERSES)
@pytest.mark.parametrize("n", SIZES)
def test_uniform_sort(ds, U, n):
    keys = w.as_u32(w.uniform(n, U, SEED + n + U))
    assert_parity(ds, keys, U, label="uniform")


@pytest.mark.parametrize("U", [6, 1000, 32768, 65536, (1 << 20) + 1, (1 << 24) + 3])
@pytest.mark.parametrize("n", [0, 777, 300_001])
def test_uniform_histogram_only(ds, U, n):
    keys = w.as_u32(w.uniform(n, U, SEED + 1 + n))
    assert_parity(ds, keys, U, mode="hist", label="uniform")


@pytest.mark.parametrize("dist", sorted(w.PAPER_DISTRIBUTIONS))
@pytest.mark.parametrize("U", [256, 1024, 65536, 1 << 18])
def test_paper_distributions(ds, dist, U):
    keys = w.as_u32(w.PAPER_DISTRIBUTIONS[dist](200_003, U, SEED))
    assert_parity(ds, keys, U, label=dist)


@pytest.mark.parametrize("U", [1, 7, 4096, 40001, 65535, 65536, (1 << 20) + 1])
@pytest.mark.parametrize("which", ["zero", "top", "mid"])
def test_all_keys_equal(ds, U, which):
    # 2^22 + 5 equal keys: one LDS16 workgroup sees far more than 65535 copies,
    # so the packed counters wrap many times
    n = (1 << 22) + 5
    k = {"zero": 0, "top": U - 1, "mid": U // 2}[which]
    keys = np.full(n, k, dtype=np.uint32)
    assert_parity(ds, keys, U, label=f"all-equal {which}")


@pytest.mark.parametrize("U,n", [(7, 4194048), (4097, 4194048), (30000, 16776192), (65535, 8388096),
                                 (65536, 8388096)])
@pytest.mark.parametrize("which", ["one", "pair"])
def test_sixteen_bit_rows_at_the_limit(ds, U, n, which):
    # slabs of 65532 keys (n = 65532 x workgroups for each ingestion kind): a
    # slab of fewer than 2^16 keys is written as a row of 16-bit counts, so
    # one bin holding the whole slab, or two bins of one packed word sharing
    # it, are the largest counts such a row ever holds
    if which == "one":
        keys = np.full(n, U - 1, dtype=np.uint32)
    else:
        b0 = (U - 2) & ~1  # bins b0 and b0 + 1 share a packed word
        keys = np.where(np.arange(n) % 2 == 0, b0, b0 + 1).astype(np.uint32)
    assert_parity(ds, keys, U, label=f"16-bit rows {which}")
    assert_parity(ds, keys, U, mode="hist", label=f"16-bit rows {which}")


@pytest.mark.parametrize("U", [4096, 40001, 65536, 1 << 24])
def test_hot_zipf(ds, U):
    keys = w.as_u32(w.hot_zipf(1_000_003, U, SEED))
    assert_parity(ds, keys, U, label="hot+zipf")


@pytest.mark.parametrize("U", [1000, 65536, (1 << 20) + 1])
def test_in_place(ds, U):
    keys = w.as_u32(w.uniform(123_457, U, SEED + 5))
    assert_parity(ds, keys, U, in_place=True, label="in-place")


@pytest.mark.parametrize("U", [1000, 40001, 65536, (1 << 20) + 1])
def test_unaligned_pointers(ds, U):
    dev = torch.device("cuda:0")
    n = 100_003
    keys_h = w.as_u32(w.uniform(n, U, SEED + 9))
    big = torch.zeros(n + 8, dtype=torch.int32, device=dev)
    keys = big[1:n + 1]
    keys.copy_(torch.from_numpy(keys_h.view(np.int32)))
    Hb = torch.zeros(U + 8, dtype=torch.int32, device=dev)
    H = Hb[3:U + 3]
    ob = torch.zeros(n + 8, dtype=torch.int32, device=dev)
    out = ob[2:n + 2]
    ws_t = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT) + 64, dev)
    ws = ws_t[17:]  # an unaligned workspace pointer is aligned up inside the library
    say(f"unaligned n={n} U={U}")
    ds.check(ds.dialsort_sort(keys, U, H, out, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    st, H_ref, out_ref = oracle.sort(keys_h, U)
    assert np.array_equal(w.as_u32(H), H_ref)
    assert np.array_equal(w.as_u32(out), out_ref)
    assert int(ob[0]) == 0 and int(ob[1]) == 0 and int(ob[n + 2]) == 0  # nothing written outside out


@pytest.mark.parametrize("U", [6, 4097, 65536, (1 << 20) + 1])
def test_key_out_of_range(ds, U):
    dev = torch.device("cuda:0")
    keys = w.uniform(50_000, U, SEED)
    keys[12345] = U  # one key == U
    say(f"erange U={U}")
    st, _, _ = gpu_sort(ds, keys.to(dev), U)
    assert st == ds.DIALSORT_ERANGE
    st, _, _ = gpu_sort(ds, keys.to(dev), U, mode="hist")
    assert st == ds.DIALSORT_ERANGE
    # the next call on a fresh workspace is clean again
    st, _, _ = gpu_sort(ds, w.uniform(1000, U, 1).to(dev), U)
    assert st == ds.DIALSORT_OK


def test_workspace_reuse_clears_state(ds):
    dev = torch.device("cuda:0")
    U = 65536
    ws = ds.workspace(ds.dialsort_workspace_bytes(1 << 20, U, ds.DIALSORT_MODE_SORT), dev)
    H = torch.empty(U, dtype=torch.int32, device=dev)
    for i, n in enumerate([1 << 20, 1000, 1 << 19]):
        keys = w.uniform(n, U, SEED + i).to(dev)
        if i == 1:
            keys[3] = U + 5
        out = torch.empty(n, dtype=torch.int32, device=dev)
        say(f"reuse call {i} n={n}")
        ds.check(ds.dialsort_sort(keys, U, H, out, ws))
        st = ds.dialsort_status_sync(ws)
        if i == 1:
            assert st == ds.DIALSORT_ERANGE
            continue
        assert st == ds.DIALSORT_OK
        _, H_ref, out_ref = oracle.sort(w.as_u32(keys), U)
        assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)


@pytest.mark.parametrize("U", [1, 6, 1000, 65536, 300_000, 1 << 24])
@pytest.mark.parametrize("shape", ["sparse", "dense", "hot"])
def test_reconstruct(ds, U, shape):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(U + len(shape))
    if shape == "sparse":
        H = (rng.random(U) < 0.05).astype(np.uint32) * rng.integers(1, 4, U).astype(np.uint32)
    elif shape == "dense":
        H = rng.integers(0, 9, U).astype(np.uint32)
    else:
        H = np.zeros(U, dtype=np.uint32)
        H[rng.integers(0, U)] = 300_000
        H[rng.integers(0, U, 50)] += 7
    total = int(H.sum(dtype=np.uint64))
    Hd = torch.from_numpy(H.view(np.int32)).to(dev)
    for cap in sorted({total, max(total - 3, 0), total // 2, total + 100}):
        out = torch.full((max(cap, 1),), -3, dtype=torch.int32, device=dev)
        ws = ds.workspace(ds.dialsort_workspace_bytes(cap, U, ds.DIALSORT_MODE_RECONSTRUCT), dev)
        say(f"reconstruct U={U} shape={shape} total={total} cap={cap}")
        ds.check(ds.dialsort_reconstruct(Hd, out, ws, out_cap=cap))
        st = ds.dialsort_status_sync(ws)
        ost, ref = oracle.reconstruct(H, cap)
        assert st == (ds.DIALSORT_EOVERFLOW if total > cap else ds.DIALSORT_OK)
        assert ost == (oracle.EOVERFLOW if total > cap else oracle.OK)
        got = w.as_u32(out)
        assert np.array_equal(got[:ref.size], ref)
        assert np.all(got[ref.size:cap] == np.uint32(0xFFFFFFFD))  # untouched beyond sum(H)
        st2, tot = ds.dialsort_result_total(ws)
        assert st2 == ds.DIALSORT_OK and tot == total


def test_universe_2_pow_32(ds):
    """U = 2^32 (the largest universe): keys anywhere in uint32.  H has 2^32 bins
    (16 GiB); it is checked on the device at the keys and by its nonzero count."""
    dev = torch.device("cuda:0")
    U = 1 << 32
    keys_h = np.array([0xFFFFFFFF, 0, 0x80000000, 0xFFFFFFFF, 12345, 0x80000000, 0xFFFFFFFE],
                      dtype=np.uint32)
    keys = torch.from_numpy(keys_h.view(np.int32)).to(dev)
    say("U = 2^32")
    st, H, out = gpu_sort(ds, keys, U)
    assert st == ds.DIALSORT_OK
    assert np.array_equal(w.as_u32(out), np.sort(keys_h))
    uniq, cnt = np.unique(keys_h, return_counts=True)
    idx = torch.from_numpy(uniq.astype(np.int64)).to(dev)
    assert w.as_u32(H[idx]).tolist() == cnt.tolist()
    assert int(torch.count_nonzero(H)) == uniq.size
    del H
    torch.cuda.empty_cache()


@pytest.mark.parametrize("U", [4096, 30000, 65536])
def test_one_launch_sort_workspace_reuse(ds, U):
    """Small LDS sorts run as one launch whose scan blocks wait for flags that
    carry the launch's epoch.  One workspace serves sorts of different sizes in
    turn (so flags of earlier launches, with other epochs and other row counts,
    are in it), and every result is exact."""
    dev = torch.device("cuda:0")
    sizes = [1 << 20, 65539, 1 << 18, 1 << 20, 300_007, 1 << 16]
    ws = ds.workspace(max(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT) for n in sizes), dev)
    for i, n in enumerate(sizes):
        kh = w.as_u32(w.uniform(n, U, SEED + 11 * i + U))
        keys = torch.from_numpy(kh.view(np.int32)).to(dev)
        H = torch.full((U,), -1, dtype=torch.int32, device=dev)
        out = torch.full((n,), -7, dtype=torch.int32, device=dev)
        say(f"one-launch reuse U={U} n={n}")
        ds.check(ds.dialsort_sort(keys, U, H, out, ws))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
        _, H_ref, out_ref = oracle.sort(kh, U)
        assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)


@pytest.mark.parametrize("U,n", [(4096, 200_000), (40001, 1 << 20), (65536, 1 << 20), (65536, (1 << 22) - 4)])
@pytest.mark.parametrize("which", ["one", "two_slices"])
def test_one_launch_sort_skew(ds, U, n, which):
    """The one-launch sort on skewed keys: every key in one bin, or split
    between the last bin of one slice of 256 bins and the first of the next."""
    if which == "one":
        keys = np.full(n, U // 3, dtype=np.uint32)
    else:
        keys = np.where(np.arange(n) % 3 == 0, 255, 256).astype(np.uint32)
    assert_parity(ds, keys, U, label=f"one-launch skew {which}")


@pytest.mark.parametrize("U,n,one", [(65536, 1 << 20, True), (2001, 50_000, True), (6, 16384, True),
                                     (65536, (1 << 22) + 5, False), (4096, 1 << 20, False)])
def test_small_sort_launches(ds, U, n, one):
    """Which launch sequence a sort takes: one k_sort_lds for a small sort
    with 16-bit rows and few keys per slice, the counting launch and the scan
    otherwise; the result is exact either way."""
    import ctypes

    import bench

    hip = bench.HipEvents()
    ev = hip.make(8)
    count = ctypes.c_uint32(0)
    kh = w.as_u32(w.uniform(n, U, SEED + n))
    keys = torch.from_numpy(kh.view(np.int32)).to("cuda:0")
    H = torch.empty(U, dtype=torch.int32, device="cuda:0")
    out = torch.empty(n, dtype=torch.int32, device="cuda:0")
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT), keys.device)
    say(f"launch sequence U={U} n={n}")
    ds.check(ds.dialsort_set_launch_events(ev, 8, count))
    try:
        ds.check(ds.dialsort_sort(keys, U, H, out, ws))
    finally:
        ds.dialsort_set_launch_events(None, 0, None)
    torch.cuda.synchronize()
    names = [ds.dialsort_launch_name(i) for i in range(count.value)]
    hip.free(ev)
    if one:
        assert len(names) == 1 and "k_sort_lds" in names[0], names
    else:
        assert not any("k_sort_lds" in x for x in names) and any("k_scan" in x for x in names), names
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    _, H_ref, out_ref = oracle.sort(kh, U)
    assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)


@pytest.mark.parametrize("U", [1, 2, 6, 128, 255, 256, 257, 1000])
@pytest.mark.parametrize("n", [5003, 16384])
def test_one_launch_sort_small_universes(ds, U, n):
    """Universes of at most a few slices of 256 bins, where the one-launch sort
    has a single slice (or a partial last one) and its rows hold few words."""
    keys = w.as_u32(w.uniform(n, U, SEED + 7 * n + U))
    assert_parity(ds, keys, U, label="one-launch small universe")


@pytest.mark.parametrize("U", [4096, 65536])
def test_single_sort_graph_capture_replay(ds, U):
    """A sort captured in a HIP graph (the launch sequence that does not rely
    on a per-launch epoch) replays exactly, several times, on new keys."""
    dev = torch.device("cuda:0")
    n = 1 << 20
    keys = torch.empty(n, dtype=torch.int32, device=dev)
    H = torch.empty(U, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT), dev)
    say(f"graph capture of one sort U={U}")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ds.check(ds.dialsort_sort(keys, U, H, out, ws, stream=side))
    torch.cuda.current_stream().wait_stream(side)
    for r in range(3):
        kh = w.as_u32(w.uniform(n, U, SEED + 100 * r + U))
        keys.copy_(torch.from_numpy(kh.view(np.int32)))
        H.fill_(-1)
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
        _, H_ref, out_ref = oracle.sort(kh, U)
        assert np.array_equal(w.as_u32(H), H_ref), f"replay {r}: H"
        assert np.array_equal(w.as_u32(out), out_ref), f"replay {r}: out"


def test_batched_equals_single(ds):
    dev = torch.device("cuda:0")
    spec = w.batch_spec(count=48, n_hi=1 << 16)
    arrays, refs = [], []
    for s in spec:
        kh = w.as_u32(s.keys())
        k = torch.from_numpy(kh.view(np.int32)).to(dev)
        arrays.append((k, s.U, torch.full((s.U,), -1, dtype=torch.int32, device=dev),
                       torch.full((s.n,), -1, dtype=torch.int32, device=dev)))
        refs.append(oracle.sort(kh, s.U))
    descs = ds.make_descs(arrays)
    ws = ds.workspace(ds.dialsort_batched_workspace_bytes(descs, len(arrays)), dev)
    say(f"batched {len(arrays)} arrays")
    ds.check(ds.dialsort_sort_batched(descs, len(arrays), ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    for (k, U, H, o), (st, H_ref, out_ref) in zip(arrays, refs):
        assert st == oracle.OK
        assert np.array_equal(w.as_u32(H), H_ref)
        assert np.array_equal(w.as_u32(o), out_ref)


@pytest.mark.parametrize("U", [1000, 4096, 40001, 65536])
def test_changing_hot_keys(ds, U):
    """Runs of different hot keys one after another, three hot keys shuffled
    together, and an alternating pair: the wave's candidate counts are replaced
    (flushed) many times and reach the flush threshold, on every LDS path."""
    rng = np.random.default_rng(U + 31)
    blocks = []
    for j in range(12):  # 12 runs of ~350K keys, each mostly one key
        b = rng.integers(0, U, 350_001).astype(np.uint32)
        b[rng.random(b.size) < 0.8] = (j * 7919) % U
        blocks.append(b)
    three = np.array([3 % U, (U // 2) | 1, U - 1], dtype=np.uint32)[rng.integers(0, 3, 1_500_000)]
    alt = np.tile(np.array([1 % U, (U - 2) % U], dtype=np.uint32), 400_000)
    keys = np.concatenate(blocks + [three, alt])
    assert_parity(ds, keys, U, label="changing hot keys")
    assert_parity(ds, keys, U, mode="hist", label="changing hot keys")


@pytest.mark.parametrize("U", [300, 4096, 32768, 65536])
def test_runs_near_window_sizes(ds, U):
    """Sorts small enough for the scan tiles to write the output themselves:
    runs of 63..70000 copies next to short ones, so that steps with only short
    runs, steps with a long one and runs across several windows all occur."""
    rng = np.random.default_rng(U + 41)
    base = rng.integers(0, U, 400_000).astype(np.uint32)
    extra = [np.full(c, (97 * i + 5) % U, dtype=np.uint32)
             for i, c in enumerate([63, 64, 65, 66, 255, 256, 257, 1000, 4099, 70000])]
    keys = np.concatenate([base] + extra)
    rng.shuffle(keys)
    assert_parity(ds, keys, U, label="runs near window sizes")
    assert_parity(ds, keys, U, in_place=True, label="runs near window sizes")


@pytest.mark.parametrize("U", [4096, 30000, 65536])
def test_range_report_through_partial_rows(ds, U):
    """n = 2^20 ingests into many partial rows, with no clearing launch first:
    each ingestion workgroup reports a key past U in its own row and the scan
    folds the reports into the status.  A bad key in the first or the last
    workgroup's slab is reported, in sort and histogram mode, and the next
    clean call on the same workspace is clean and exact again."""
    dev = torch.device("cuda:0")
    n = 1 << 20
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT), dev)
    H = torch.empty(U, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    for pos in [0, n - 1]:
        keys = w.uniform(n, U, SEED + pos).to(dev)
        keys[pos] = U + pos % 7
        say(f"range report U={U} pos={pos}")
        ds.check(ds.dialsort_sort(keys, U, H, out, ws))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_ERANGE
        ds.check(ds.dialsort_histogram(keys, U, H, ws))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_ERANGE
        good = w.uniform(n, U, SEED + 3 + pos).to(dev)
        ds.check(ds.dialsort_sort(good, U, H, out, ws))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
        _, H_ref, out_ref = oracle.sort(w.as_u32(good), U)
        assert np.array_equal(w.as_u32(H), H_ref) and np.array_equal(w.as_u32(out), out_ref)


@pytest.mark.parametrize("case", ["one_hot_whole_bucket", "one_hot_split_bucket", "three_hot_fields_wrap",
                                  "many_runs"])
def test_partitioned_hot_keys(ds, case):
    """Partitioned path (U = 2^20 + 1, buckets of 2^16 bins) with keys whose
    counts pass 2^16 inside one bucket.  The bucket pass counts each wave's
    hot key in registers: a whole bucket reads such a bin through its hot
    table, a part of a split bucket adds the table into the scratch row, and
    a bucket whose other keys still wrap a 16-bit field is counted again in
    halves.  The last case, 400 keys of one bucket in runs of equal keys,
    makes the candidates change often."""
    rng = np.random.default_rng(SEED + ["one_hot_whole_bucket", "one_hot_split_bucket", "three_hot_fields_wrap",
                                        "many_runs"].index(case))
    U = (1 << 20) + 1
    if case == "one_hot_whole_bucket":
        # 200 000 copies of one key; its bucket stays whole (below 2 chunks)
        keys = rng.integers(0, U, 400_000).astype(np.uint32)
        keys = np.concatenate([keys, np.full(200_000, 3 * 65536 + 777, dtype=np.uint32)])
    elif case == "one_hot_split_bucket":
        # 2 million copies of one key: its bucket is split into parts, each
        # holding far more than 2^16 copies
        keys = rng.integers(0, U, 1_000_000).astype(np.uint32)
        keys = np.concatenate([keys, np.full(2_000_000, 9 * 65536 + 12345, dtype=np.uint32)])
    elif case == "three_hot_fields_wrap":
        # three keys of 150 000 copies each in one whole bucket: a wave has one
        # candidate, so the others' 16-bit fields wrap
        keys = rng.integers(0, U, 300_000).astype(np.uint32)
        hot = [5 * 65536 + 1, 5 * 65536 + 2, 5 * 65536 + 60000]
        keys = np.concatenate([keys] + [np.full(150_000, h, dtype=np.uint32) for h in hot])
    else:
        # 400 keys of one bucket in runs of 1500 equal keys, in order
        runs = [np.full(1500, 7 * 65536 + 97 * i, dtype=np.uint32) for i in range(400)]
        keys = np.concatenate([rng.integers(0, U, 100_000).astype(np.uint32)] + runs)
    if case != "many_runs":
        rng.shuffle(keys)
    assert_parity(ds, keys, U, label=case)
    assert_parity(ds, keys, U, mode="hist", label=case)


@pytest.mark.parametrize("dist", ["sorted", "reverse"])
@pytest.mark.parametrize("U", [4096, 40001, 65536])
def test_sorted_runs_large(ds, dist, U):
    """2^24 sorted or reverse-sorted keys: every lane's 16-byte load holds a
    run of equal keys, merged in the lane before the wave merge, on the
    32-bit and the packed 16-bit LDS paths."""
    keys = w.as_u32(w.PAPER_DISTRIBUTIONS[dist](1 << 24, U, SEED + 5))
    assert_parity(ds, keys, U, label=f"{dist} 2^24")
    assert_parity(ds, keys, U, mode="hist", label=f"{dist} 2^24")
