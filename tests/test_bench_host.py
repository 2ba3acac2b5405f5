"""Host-side checks of the benchmark's accounting: the algorithmic bytes each
kernel is credited with (ingestion reads every key once and H is written once,
Eq. (1); the projection reads H once and writes the output, Eq. (2)), the
source digest the committed counter summary is keyed to, and the traffic
lookup that reads that summary."""

from __future__ import annotations

import os
import re

import bench

N, U = 10**8, 1 << 24


def test_algo_bytes_per_kernel():
    assert bench.algo_bytes("(k_partition<1024, 3, true>)", N, U, "sort") == 4 * N
    assert bench.algo_bytes("(k_hist_lds<1024, 32768, true, 3, true, 4>)", N, U, "hist") == 4 * N
    assert bench.algo_bytes("(k_bucket<3, true, true>)", N, U, "sort") == 4 * U
    assert bench.algo_bytes("(k_scan<SCAN_NT, 1, true>)", N, U, "sort") == 4 * U
    for name in ("(k_fill<FILL_NT, FILL_CL2, true>)", "(k_fill<FILL_NT, FILL_CL2, true, false, true>)"):
        assert bench.algo_bytes(name, N, U, "sort") == 4 * N + 4 * U
        assert bench.algo_bytes(name, N, U, "hist") == 0
    assert bench.algo_bytes("k_init", N, U, "sort") == 0


def test_kernels_of_one_sort_add_up_to_the_path():
    # partitioned path: 8 B per key plus 8 B per bin in all
    names = ("k_init", "(k_partition<1024, 3, true>)", "(k_bucket<3, true, true>)",
             "(k_fill<FILL_NT, FILL_CL2, true, false, true>)")
    assert sum(bench.algo_bytes(k, N, U, "sort") for k in names) == 8 * N + 8 * U
    # histogram only: 4 B per key plus 4 B per bin
    names = ("k_init", "(k_partition<1024, 3, true>)", "(k_bucket<3, true, false>)")
    assert sum(bench.algo_bytes(k, N, U, "hist") for k in names) == 4 * N + 4 * U


def test_source_digest_is_stable_and_depends_on_the_sources():
    d = bench.source_digest()
    assert re.fullmatch(r"[0-9a-f]{64}", d)
    assert d == bench.source_digest()
    assert bench.source_digest("radix.hip") != d


def test_traffic_lookup_matches_the_summary_it_reads():
    with open(os.path.join(bench.ROOT, "profiles", "large_uniform_sort_counters.txt")) as f:
        m = re.search(r"# source-sha256: ([0-9a-f]{64})", f.read())
    assert m, "the counter summary records the digest of the sources it was taken on"
    t = bench.profiled_traffic("(k_bucket<3, true, true>)")
    if m.group(1) != bench.source_digest():
        assert t is None  # a stale summary reports no traffic
        return
    assert t is not None
    assert abs(t["bytes"] - t["fetch_bytes"] - t["write_bytes"]) < 1.0
    # the bucket pass reads at least the staging (2 B per key) and writes at least H
    assert t["fetch_bytes"] >= 2 * N and t["write_bytes"] >= 4 * U
    assert bench.profiled_traffic("(k_no_such_kernel<1>)") is None
