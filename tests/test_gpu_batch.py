"""GPU parity of the batched path: the fused persistent launch (every autotuner
configuration), the per-array form, the autotuner, HIP-graph capture and
replay, against the CPU oracle, bit-exact for every array of the batch.

The mixed batch holds the uneven-batch recipe at small sizes plus the edge
arrays of the fused form: no keys, U = 1, non-power-of-two U, U just above and
below the LDS width, one key repeated past the 16-bit packed counter range,
many buckets (U = 2^22), a tiny n next to a large U, and arrays sorted in place.
"""

from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
CONFIGS = [(nt, lw, ch) for nt in (512, 1024) for lw in (14, 15, 16) for ch in (1 << 18, 1 << 20, 1 << 22)]


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ds(cuda):
    import paper_2605_16667_amd as m

    return m


class Batch:
    """Device arrays of a batch plus the oracle's answers."""

    def __init__(self, ds, specs):
        self.items = []
        for i, (kh, U, in_place) in enumerate(specs):
            k = torch.from_numpy(kh.view(np.int32).copy()).to(DEV)
            H = torch.empty(U, dtype=torch.int32, device=DEV)
            out = k if in_place else torch.empty(kh.size, dtype=torch.int32, device=DEV)
            st, H_ref, out_ref = oracle.sort(kh, U)
            assert st == oracle.OK
            self.items.append((k, U, H, out, H_ref, out_ref, in_place))
        self.descs = ds.make_descs([(k, U, H, o) for (k, U, H, o, *_r) in self.items])
        self.count = len(self.items)
        self.ws = ds.workspace(ds.dialsort_batched_workspace_bytes(self.descs, self.count), DEV)

    def poison(self):
        for (k, U, H, out, _h, _o, in_place) in self.items:
            H.fill_(-1)
            if not in_place:
                out.fill_(-7)

    def check(self, label):
        torch.cuda.synchronize()
        for i, (k, U, H, out, H_ref, out_ref, _ip) in enumerate(self.items):
            Hh = w.as_u32(H)
            if not np.array_equal(Hh, H_ref):
                bad = np.nonzero(Hh != H_ref)[0]
                raise AssertionError(f"{label}: array {i} (n={out_ref.size}, U={U}) H differs at {bad.size} bins, "
                                     f"first {bad[:4]}: {Hh[bad[:4]]} vs {H_ref[bad[:4]]}")
            oh = w.as_u32(out)
            if not np.array_equal(oh, out_ref):
                bad = np.nonzero(oh != out_ref)[0]
                raise AssertionError(f"{label}: array {i} (n={out_ref.size}, U={U}) out differs at {bad.size} "
                                     f"positions, first {bad[:4]}")


BARRAY_BYTES = 120  # sizeof(BArray) in the workspace tables
BSTATE_BYTES = 32


def raw_status(batch):
    """The batch's raw device status word and the nonzero per-array status
    words, for failure messages."""
    torch.cuda.synchronize()
    ws = batch.ws
    word = int(ws[:4].view(torch.int32).item()) & 0xFFFFFFFF
    off = (256 + batch.count * BARRAY_BYTES + 255) // 256 * 256
    st = ws[off:off + batch.count * BSTATE_BYTES].view(torch.int32).view(batch.count, 8).cpu().numpy()
    bad = [(i, hex(int(st[i, 6]) & 0xFFFFFFFF), batch.items[i][5].size, batch.items[i][1])
           for i in range(batch.count) if st[i, 6] != 0]
    return f"status word {word:#x}; arrays (index, status, n, U): {bad}"


def mixed_specs(seed_shift=0):
    rng = np.random.default_rng(w.BASE_SEED + 50 + seed_shift)
    specs = []
    for s in w.batch_spec(count=40, n_hi=1 << 17, seed=w.BASE_SEED + 3 + seed_shift):
        specs.append((w.as_u32(s.keys()), s.U, False))

    def uni(n, U):
        return rng.integers(0, U, n, dtype=np.uint64).astype(np.uint32)

    specs += [
        (np.zeros(0, np.uint32), 5, False),
        (np.zeros(1, np.uint32), 1, False),
        (uni(7, 3), 3, False),
        (uni(1000, 366), 366, False),
        (uni(70001, 1 << 14), 1 << 14, False),
        (uni(70002, (1 << 14) + 1), (1 << 14) + 1, False),
        (uni(90003, 1 << 16), 1 << 16, False),
        (uni(90004, (1 << 16) + 1), (1 << 16) + 1, False),
        (np.full(300001, 40000 - 3, np.uint32), 40000, False),
        (uni(200005, 1 << 22), 1 << 22, False),
        (uni(5, 1 << 20), 1 << 20, False),
        (uni(123457, 1 << 12), 1 << 12, True),
        (uni(54321, 1 << 19), 1 << 19, True),
    ]
    return specs


@pytest.fixture(scope="module")
def batch(ds):
    return Batch(ds, mixed_specs())


@pytest.mark.parametrize("cfg", CONFIGS, ids=[f"nt{c[0]}-w{c[1]}-c{c[2].bit_length() - 1}" for c in CONFIGS])
def test_fused_every_config(ds, batch, cfg):
    say(f"fused batch of {batch.count} arrays, config {cfg}")
    batch.poison()
    st, plan = ds.dialsort_batch_prepare(batch.descs, batch.count, ds.batch_config(*cfg), batch.ws)
    ds.check(st)
    assert plan.units > 0 and plan.grid > 0
    ds.check(ds.dialsort_batch_launch(plan))
    st = ds.dialsort_status_sync(batch.ws)
    assert st == ds.DIALSORT_OK, raw_status(batch)
    batch.check(f"config {cfg}")
    # a second launch of the same plan recomputes everything
    batch.poison()
    ds.check(ds.dialsort_batch_launch(plan))
    st = ds.dialsort_status_sync(batch.ws)
    assert st == ds.DIALSORT_OK, raw_status(batch)
    batch.check(f"config {cfg}, relaunch")


def test_per_array_form(ds, batch):
    say("per-array launches (dialsort_sort_each)")
    batch.poison()
    ds.check(ds.dialsort_sort_each(batch.descs, batch.count, batch.ws))
    assert ds.dialsort_status_sync(batch.ws) == ds.DIALSORT_OK
    batch.check("sort_each")


def test_autotune_then_default(ds, batch):
    say("autotune")
    st, best = ds.dialsort_batch_autotune(batch.descs, batch.count, batch.ws)
    ds.check(st)
    assert (best.block, best.log2_width, best.chunk_keys) in CONFIGS
    st, dflt = ds.dialsort_batch_default_config(batch.descs, batch.count)
    ds.check(st)
    assert (dflt.block, dflt.log2_width, dflt.chunk_keys) == (best.block, best.log2_width, best.chunk_keys)
    batch.poison()
    ds.check(ds.dialsort_sort_batched(batch.descs, batch.count, batch.ws))
    assert ds.dialsort_status_sync(batch.ws) == ds.DIALSORT_OK
    batch.check("sort_batched after autotune")


def test_graph_capture_replay(ds, batch):
    say("graph capture of the fused launch, 3 replays")
    st, plan = ds.dialsort_batch_prepare(batch.descs, batch.count, ds.batch_config(1024, 16, 1 << 20), batch.ws)
    ds.check(st)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ds.check(ds.dialsort_batch_launch(plan, stream=side))
    torch.cuda.current_stream().wait_stream(side)
    for r in range(3):
        batch.poison()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ds.dialsort_status_sync(batch.ws) == ds.DIALSORT_OK
        batch.check(f"graph replay {r}")


def test_batch_times(ds, batch):
    say("per-array completion times")
    st, plan = ds.dialsort_batch_prepare(batch.descs, batch.count, None, batch.ws)
    ds.check(st)
    ds.check(ds.dialsort_batch_launch(plan))
    st, times, total = ds.dialsort_batch_times(plan, batch.count)
    ds.check(st)
    assert total > 0
    assert all(0 <= t <= total * 1.0001 + 1e-6 for t in times)
    assert max(times) == pytest.approx(total, rel=1e-3, abs=1e-4)


def test_key_out_of_range_in_one_array(ds):
    rng = np.random.default_rng(7)
    specs = [(rng.integers(0, 1000, 5000).astype(np.uint32), 1000, False) for _ in range(3)]
    bad = rng.integers(0, 1 << 18, 40000).astype(np.uint32)
    bad[12345] = 1 << 18  # == U
    specs.append((bad, 1 << 18, False))
    say("ERANGE in one array of four")
    k = [torch.from_numpy(s[0].view(np.int32).copy()).to(DEV) for s in specs]
    arrays = [(k[i], specs[i][1], torch.empty(specs[i][1], dtype=torch.int32, device=DEV),
               torch.empty(specs[i][0].size, dtype=torch.int32, device=DEV)) for i in range(4)]
    descs = ds.make_descs(arrays)
    ws = ds.workspace(ds.dialsort_batched_workspace_bytes(descs, 4), DEV)
    for cfg in [(1024, 16, 1 << 20), (512, 14, 1 << 18)]:
        st, plan = ds.dialsort_batch_prepare(descs, 4, ds.batch_config(*cfg), ws)
        ds.check(st)
        ds.check(ds.dialsort_batch_launch(plan))
        assert ds.dialsort_status_sync(ws) == ds.DIALSORT_ERANGE
    ds.check(ds.dialsort_sort_each(descs, 4, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_ERANGE


def test_unaligned_array_falls_back(ds):
    rng = np.random.default_rng(8)
    kh = rng.integers(0, 5000, 20001).astype(np.uint32)
    base = torch.from_numpy(np.concatenate([[0], kh]).astype(np.uint32).view(np.int32)).to(DEV)
    k = base[1:]  # 4 bytes past a 256-byte boundary
    H = torch.empty(5000, dtype=torch.int32, device=DEV)
    out = torch.empty(kh.size, dtype=torch.int32, device=DEV)
    k2h = rng.integers(0, 1 << 17, 30000).astype(np.uint32)
    k2 = torch.from_numpy(k2h.view(np.int32)).to(DEV)
    H2 = torch.empty(1 << 17, dtype=torch.int32, device=DEV)
    out2 = torch.empty(k2h.size, dtype=torch.int32, device=DEV)
    descs = ds.make_descs([(k, 5000, H, out), (k2, 1 << 17, H2, out2)])
    ws = ds.workspace(ds.dialsort_batched_workspace_bytes(descs, 2), DEV)
    say("batch with a misaligned array: prepare refuses, sort_batched falls back")
    st, _plan = ds.dialsort_batch_prepare(descs, 2, None, ws)
    assert st == ds.DIALSORT_EINVAL
    ds.check(ds.dialsort_sort_batched(descs, 2, ws))
    assert ds.dialsort_status_sync(ws) == ds.DIALSORT_OK
    for (kk, U, HH, oo) in [(kh, 5000, H, out), (k2h, 1 << 17, H2, out2)]:
        _s, H_ref, out_ref = oracle.sort(kk, U)
        assert np.array_equal(w.as_u32(HH), H_ref)
        assert np.array_equal(w.as_u32(oo), out_ref)


def test_batch_spec_workload_sample(ds):
    """A 256-array sample of the uneven-batch recipe at full per-array sizes
    (n up to 2^22, U up to 2^20), fused with the default configuration."""
    specs = [(w.as_u32(s.keys()), s.U, False) for s in w.batch_spec(count=4096)[:256]]
    b = Batch(ds, specs)
    say(f"uneven-batch sample: {b.count} arrays, {sum(s[0].size for s in specs)} keys")
    b.poison()
    st, plan = ds.dialsort_batch_prepare(b.descs, b.count, None, b.ws)
    ds.check(st)
    ds.check(ds.dialsort_batch_launch(plan))
    assert ds.dialsort_status_sync(b.ws) == ds.DIALSORT_OK
    b.check("uneven-batch sample")
