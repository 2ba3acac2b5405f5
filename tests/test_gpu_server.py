"""GPU tests of the serving engine: every request's H and output equal the
oracle's and equal the result of the same request served alone, whatever else
shares its batch; admission by arena footprint; per-request errors; release
and drain rules."""

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


def make_server(ds, arena_bytes, max_inflight=2, max_batch=64, cfg=(1024, 16, 1 << 20)):
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=DEV)
    st, srv = ds.dialsort_server_create(arena, ds.server_config(ds.batch_config(*cfg), max_inflight, max_batch))
    ds.check(st)
    return arena, srv


def result(ds, arena, srv, rid):
    st, info = ds.dialsort_server_info(srv, rid)
    ds.check(st)
    assert info.state == ds.DIALSORT_REQ_DONE
    H = ds.arena_view(arena, info.H, info.U).clone()
    out = ds.arena_view(arena, info.out, info.n).clone()
    return info, H, out


def small_stream(count, seed_shift=0):
    """Requests of the served workload's recipe, at sizes the oracle checks fast."""
    reqs = w.request_stream(count, 1000.0, seed=w.BASE_SEED + 4 + seed_shift, n_lo=1 << 10, n_hi=1 << 18)
    out = []
    for r in reqs:
        kh = w.as_u32(r.spec.keys())
        out.append((kh, r.spec.U))
    return out


def test_alone_equals_in_mix(ds):
    rng = np.random.default_rng(11)
    kR = w.as_u32(w.zipf(300001, 1 << 20, 1.2, w.BASE_SEED + 77))
    keysR = torch.from_numpy(kR.view(np.int32)).to(DEV)
    st_ref, H_ref, out_ref = oracle.sort(kR, 1 << 20)
    assert st_ref == oracle.OK
    arena, srv = make_server(ds, 1 << 30)
    try:
        say("request alone")
        st, rid = ds.dialsort_server_submit(srv, keysR, 1 << 20)
        ds.check(st)
        ds.check(ds.dialsort_server_drain(srv))
        info, H_alone, out_alone = result(ds, arena, srv, rid)
        assert info.status == ds.DIALSORT_OK
        ds.check(ds.dialsort_server_release(srv, rid))
        assert np.array_equal(w.as_u32(H_alone), H_ref) and np.array_equal(w.as_u32(out_alone), out_ref)

        say("the same request in a mix of 40, submitted while batches run")
        mix = small_stream(40)
        dev_keys = [torch.from_numpy(k.view(np.int32)).to(DEV) for k, _ in mix]
        ids = []
        pos_R = 17
        for i, (k, U) in enumerate(mix):
            if i == pos_R:
                st, ridR = ds.dialsort_server_submit(srv, keysR, 1 << 20)
                ds.check(st)
            st, rid = ds.dialsort_server_submit(srv, dev_keys[i], U)
            ds.check(st)
            ids.append(rid)
            if i % 3 == 0:
                ds.check(ds.dialsort_server_poll(srv)[0])
        ds.check(ds.dialsort_server_drain(srv))
        info, H_mix, out_mix = result(ds, arena, srv, ridR)
        assert info.status == ds.DIALSORT_OK
        assert torch.equal(H_mix, H_alone) and torch.equal(out_mix, out_alone)
        launches = set()
        for (k, U), rid in zip(mix, ids):
            info, H, out = result(ds, arena, srv, rid)
            assert info.status == ds.DIALSORT_OK
            launches.add(round(info.launch_ms, 6))
            st, Hr, outr = oracle.sort(k, U)
            assert np.array_equal(w.as_u32(H), Hr)
            assert np.array_equal(w.as_u32(out), outr)
            assert info.submit_ms <= info.launch_ms + 1e-6 and info.done_ms > 0
            ds.check(ds.dialsort_server_release(srv, rid))
        ds.check(ds.dialsort_server_release(srv, ridR))
        assert len(launches) >= 2  # requests were batched as they arrived, not all at once
    finally:
        ds.check(ds.dialsort_server_destroy(srv))


def test_admission_under_small_arena(ds):
    reqs = small_stream(24, seed_shift=1)
    need = max(ds.dialsort_server_footprint(k.size, U) for k, U in reqs)
    arena_bytes = 6 * need + (64 << 20)
    say(f"24 requests through an arena of {arena_bytes >> 20} MiB")
    arena, srv = make_server(ds, arena_bytes, max_inflight=2, max_batch=8)
    try:
        dev_keys = [torch.from_numpy(k.view(np.int32)).to(DEV) for k, _ in reqs]
        ids = []
        for kd, (k, U) in zip(dev_keys, reqs):
            st, rid = ds.dialsort_server_submit(srv, kd, U)
            ds.check(st)
            ids.append(rid)
        done = set()
        batches = set()
        spins = 0
        while len(done) < len(ids):
            st, pending = ds.dialsort_server_poll(srv)
            ds.check(st)
            for (k, U), rid in zip(reqs, ids):
                if rid in done:
                    continue
                st, info = ds.dialsort_server_info(srv, rid)
                if info.state == ds.DIALSORT_REQ_DONE:
                    _i, H, out = result(ds, arena, srv, rid)
                    assert info.status == ds.DIALSORT_OK
                    batches.add(round(info.launch_ms, 6))
                    s2, Hr, outr = oracle.sort(k, U)
                    assert np.array_equal(w.as_u32(H), Hr) and np.array_equal(w.as_u32(out), outr)
                    ds.check(ds.dialsort_server_release(srv, rid))
                    done.add(rid)
            spins += 1
            assert spins < 200000
        assert len(batches) >= 3  # the arena forced several admission rounds
    finally:
        ds.check(ds.dialsort_server_destroy(srv))


def test_bad_request_does_not_spoil_its_batch(ds):
    rng = np.random.default_rng(12)
    good = [rng.integers(0, 5000, 20000).astype(np.uint32) for _ in range(3)]
    bad = rng.integers(0, 1 << 18, 30000).astype(np.uint32)
    bad[777] = 1 << 18
    arena, srv = make_server(ds, 1 << 28)
    try:
        say("one request with a key >= U among four")
        ks = [torch.from_numpy(k.view(np.int32)).to(DEV) for k in good + [bad]]
        Us = [5000, 5000, 5000, 1 << 18]
        ids = []
        for k, U in zip(ks, Us):
            st, rid = ds.dialsort_server_submit(srv, k, U)
            ds.check(st)
            ids.append(rid)
        ds.check(ds.dialsort_server_drain(srv))
        for i, rid in enumerate(ids):
            info, H, out = result(ds, arena, srv, rid)
            if i < 3:
                assert info.status == ds.DIALSORT_OK
                s2, Hr, outr = oracle.sort(good[i], 5000)
                assert np.array_equal(w.as_u32(H), Hr) and np.array_equal(w.as_u32(out), outr)
            else:
                assert info.status == ds.DIALSORT_ERANGE
    finally:
        ds.check(ds.dialsort_server_destroy(srv))


def test_release_rules_and_held_arena(ds):
    rng = np.random.default_rng(13)
    k = torch.from_numpy(rng.integers(0, 1 << 16, 1 << 20).astype(np.uint32).view(np.int32)).to(DEV)
    need = ds.dialsort_server_footprint(1 << 20, 1 << 16)
    # room for two requests' H and output; the spare MiB holds a fused launch's
    # workspace (a lone request falls back to it when dialsort_sort's does not fit)
    arena, srv = make_server(ds, 2 * need + (1 << 20), max_batch=1)
    try:
        say("errors, and a drain blocked by results that were not released")
        st, _ = ds.dialsort_server_submit(srv, k[1:], 1 << 16)  # misaligned keys
        assert st == ds.DIALSORT_EINVAL
        big = torch.empty(1 << 28, dtype=torch.int32, device=DEV)
        st, _ = ds.dialsort_server_submit(srv, big, 1 << 16)  # can never fit
        assert st == ds.DIALSORT_EWORKSPACE
        del big
        ids = []
        for _ in range(3):
            st, rid = ds.dialsort_server_submit(srv, k, 1 << 16)
            ds.check(st)
            ids.append(rid)
        assert ds.dialsort_server_release(srv, ids[2]) == ds.DIALSORT_EINVAL  # not done
        assert ds.dialsort_server_drain(srv) == ds.DIALSORT_EWORKSPACE  # two results hold the arena
        st, info = ds.dialsort_server_info(srv, ids[2])
        assert info.state == ds.DIALSORT_REQ_QUEUED
        ds.check(ds.dialsort_server_release(srv, ids[0]))
        ds.check(ds.dialsort_server_drain(srv))
        kh = w.as_u32(k)
        s2, Hr, outr = oracle.sort(kh, 1 << 16)
        for rid in ids[1:]:
            info, H, out = result(ds, arena, srv, rid)
            assert np.array_equal(w.as_u32(H), Hr) and np.array_equal(w.as_u32(out), outr)
        assert ds.dialsort_server_info(srv, ids[0])[0] == ds.DIALSORT_EINVAL  # released
    finally:
        ds.check(ds.dialsort_server_destroy(srv))


def test_queries_on_resident_histograms(ds):
    """Served requests keep H in the arena until they are released; the queries
    of the canonical ordered state (Sec. 3.3) run on it there, through a view of
    the arena (nothing is copied), and match the oracle on the request's keys."""
    reqs = small_stream(12, seed_shift=3)
    dev_keys = [torch.from_numpy(k.view(np.int32)).to(DEV) for k, _ in reqs]
    arena, srv = make_server(ds, 1 << 30)
    try:
        ids = []
        for kd, (_, U) in zip(dev_keys, reqs):
            st, rid = ds.dialsort_server_submit(srv, kd, U)
            ds.check(st)
            ids.append(rid)
        ds.check(ds.dialsort_server_drain(srv))
        rng = np.random.default_rng(17)
        for rid, (kh, U) in zip(ids, reqs):
            st, info = ds.dialsort_server_info(srv, rid)
            ds.check(st)
            assert info.state == ds.DIALSORT_REQ_DONE and info.status == ds.DIALSORT_OK
            say(f"queries on the resident H of request {rid}: n={info.n} U={U}")
            H = ds.arena_view(arena, info.H, info.U)
            st_o, H_ref = oracle.histogram(kh, U)
            assert st_o == oracle.OK
            q = np.concatenate([rng.integers(0, U, 500), kh[:100], [U - 1, U]]).astype(np.uint32)
            qd = torch.from_numpy(q.view(np.int32)).to(DEV)
            f = torch.empty(q.size, dtype=torch.int32, device=DEV)
            ds.check(ds.dialsort_query_frequency(H, U, qd, f))
            assert np.array_equal(w.as_u32(f), oracle.frequency(H_ref, q))
            pres = torch.empty(q.size, dtype=torch.uint8, device=DEV)
            ds.check(ds.dialsort_query_presence(H, U, qd, pres))
            assert np.array_equal(pres.cpu().numpy(), oracle.presence(H_ref, q))
            P = torch.empty(U + 1, dtype=torch.int64, device=DEV)
            ws = ds.workspace(ds.dialsort_prefix_workspace_bytes(U))
            ds.check(ds.dialsort_prefix(H, U, P, ws))
            assert np.array_equal(P.cpu().numpy().view(np.uint64), oracle.prefix(H_ref))
            a = rng.integers(0, U + 1, 200).astype(np.uint64)
            b = np.minimum(a + rng.integers(0, U + 1, 200).astype(np.uint64), np.uint64(U))
            rc = torch.empty(a.size, dtype=torch.int64, device=DEV)
            ds.check(ds.dialsort_query_range_count(P, U, torch.from_numpy(a.view(np.int64)).to(DEV),
                                                   torch.from_numpy(b.view(np.int64)).to(DEV), rc))
            assert np.array_equal(rc.cpu().numpy().view(np.uint64), oracle.range_count(H_ref, a, b))
            r = np.concatenate([rng.integers(0, kh.size, 200), [0, kh.size - 1, kh.size]]).astype(np.uint64)
            sel = torch.empty(r.size, dtype=torch.int32, device=DEV)
            ds.check(ds.dialsort_query_select(P, U, torch.from_numpy(r.view(np.int64)).to(DEV), sel))
            assert np.array_equal(w.as_u32(sel), oracle.select(H_ref, r))
            # the queries left the request's H as the server wrote it
            assert np.array_equal(w.as_u32(H), H_ref)
            ds.check(ds.dialsort_server_release(srv, rid))
    finally:
        ds.check(ds.dialsort_server_destroy(srv))


def test_served_upper_sizes_match_the_oracle(ds):
    """The served workload's upper request sizes through one server: eight
    requests of n = 2^24 keys (U in {2^20, 2^24}, uniform and Zipf(1.2)) mixed
    with 24 small ones, submitted in two waves so that the second arrives while
    the first is on the device.  Every request's H and output must equal the
    oracle's (Sec. 3.3, Eqs. (1) and (2)), element by element."""
    big = []
    for j, (U, dist) in enumerate([(1 << 20, "uniform"), (1 << 24, "uniform"), (1 << 20, "zipf"), (1 << 24, "zipf")] * 2):
        spec = w.ArraySpec(1 << 24, U, dist, 1.2, w.BASE_SEED + 900 + j)
        big.append((w.as_u32(spec.keys()), U))
    small = small_stream(24, seed_shift=5)
    mix = []
    for i in range(len(small)):
        mix.append(small[i])
        if i % 3 == 1:
            mix.append(big[i // 3])
    assert sum(1 for k, _ in mix if k.size == 1 << 24) == 8
    dev_keys = [torch.from_numpy(k.view(np.int32)).to(DEV) for k, _ in mix]
    torch.cuda.synchronize()
    arena, srv = make_server(ds, 6 << 30, max_inflight=2, max_batch=64)
    try:
        ids = []
        half = len(mix) // 2
        say(f"served mix: {len(mix)} requests, 8 of n=2^24, first wave of {half}")
        for i in range(half):
            st, rid = ds.dialsort_server_submit(srv, dev_keys[i], mix[i][1])
            ds.check(st)
            ids.append(rid)
        ds.check(ds.dialsort_server_poll(srv)[0])
        say("second wave, submitted while the first runs")
        for i in range(half, len(mix)):
            st, rid = ds.dialsort_server_submit(srv, dev_keys[i], mix[i][1])
            ds.check(st)
            ids.append(rid)
            if i % 4 == 0:
                ds.check(ds.dialsort_server_poll(srv)[0])
        ds.check(ds.dialsort_server_drain(srv))
        per_launch = {}
        for (kh, U), rid in zip(mix, ids):
            info, H, out = result(ds, arena, srv, rid)
            say(f"request {rid}: n={kh.size} U={U}")
            assert info.status == ds.DIALSORT_OK
            per_launch.setdefault(round(info.launch_ms, 6), []).append(kh.size)
            st_o, Hr, outr = oracle.sort(kh, U)
            assert st_o == oracle.OK
            assert np.array_equal(w.as_u32(H), Hr), f"H of request {rid}"
            assert np.array_equal(w.as_u32(out), outr), f"output of request {rid}"
            assert info.seen_ms >= info.submit_ms
            ds.check(ds.dialsort_server_release(srv, rid))
        # some fused launch carried a request of 2^24 keys together with others
        assert any(len(v) > 1 and max(v) == 1 << 24 for v in per_launch.values())
    finally:
        ds.check(ds.dialsort_server_destroy(srv))
