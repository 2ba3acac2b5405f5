#!/usr/bin/env python3
"""DialSort hot path on one MI355X: throughput, roofline and CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workloads a,b,...] [--no-cpu]

A step is one dialsort_sort call (ingestion + ordered projection) on one batch
of synthetic keys already resident in HBM.  The headline workload is the large
uniform single sort: n = 10^8 keys uniform on [0, 2^24), U = 2^24, full
reconstruction.  Prints ONE JSON line.  Other workloads are reported as extra
fields of the same line:
  hist     the same keys, histogram-only (dialsort_histogram)
  plain    n = 2^20 uniform keys, U = 2^16 (latency of one sort)
  skewed   n = 2^28, U = 2^16, half the keys one hot value, the rest Zipf(1.2);
           beside it the same n and U with uniform keys; full sort and
           histogram-only (ingestion alone) for both
  batch    4096 uneven arrays: one autotuned fused launch replayed from a HIP
           graph, against one launch sequence per array; per-array p50/p99
  serve    a Poisson request stream through the serving engine at several
           loads, against serial plain sorts; p50/p99 latency and keys/s
  query    queries on the large workload's histogram: the running count over
           2^24 bins, and 2^20 frequency/presence/range-count/select queries
  transforms  the key transforms (offset, key range, lookup table) and
           ingestion in ten pieces at n = 1e8, U = 2^24, beside the plain forms
  windows  64 tumbling windows of 2^20 keys (U = 2^16): ingestion of one window
           overlapped with the projection of the previous one, vs one stream
  radix    DialSort-Radix over the whole signed int32 range, n = 1e7 and 1e8
The roofline object is for the kernel that takes the most time per step,
measured with HIP events recorded on the launch stream around every kernel of
every timed step (dialsort_set_launch_events).  Its algorithmic bytes are the
method's compulsory traffic that this kernel is responsible for (algo_bytes
below); its `traffic` is the HBM bytes per launch that rocprofv3 counted for
this very kernel source (profiles/large_uniform_sort_counters.txt: FETCH_SIZE
and WRITE_SIZE scaled by what they read for a plain device copy), or null when
the kernels changed since the counters were taken.  path_roofline relates the
whole step to the path's algorithmic bytes, against the 8 TB/s peak and
against the bandwidth a plain device copy reaches on the same GPU.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sorted keys/s at n=100M,U=2^24 (% HBM roofline); batched p50/p99 latency"
HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
SERVE_SLOTS = 4    # batches (or lone requests) the server keeps on the device at once


# Where the Zipf and hot-key inputs are generated before they are placed in
# device memory: "cuda" by default; "cpu" with --host-inputs (the same
# distributions from the host generator's stream; keeps the device sorts behind
# torch.randperm out of profiled runs).
GEN_DEVICE = "cuda"


def gen(t):
    """A generated input tensor, moved to the GPU if it was made on the host."""
    return t if t.is_cuda else t.to("cuda")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles created through the HIP runtime that torch has loaded."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def make(self, k):
        arr = (ctypes.c_void_p * k)()
        for i in range(k):
            ev = ctypes.c_void_p()
            if self.lib.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            arr[i] = ev
        return arr

    def ms(self, a, b):
        out = ctypes.c_float()
        if self.lib.hipEventElapsedTime(ctypes.byref(out), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return out.value

    def free(self, arr):
        for ev in arr:
            self.lib.hipEventDestroy(ev)


def algo_bytes(name: str, n: int, U: int, mode: str) -> int:
    """Compulsory bytes of the method handled by one launch of kernel `name`:
    ingestion reads the keys (4n), the histogram is written once (4U) by the
    kernel that produces it (k_bucket, or k_scan from partial rows) and, in a
    sort, read once by the projection, k_fill, which also writes the output
    (4n).  The item boundaries k_bucket and k_scan derive come from data they
    already hold.  Partial rows, staging, counters and fill items are the
    implementation's own and count against the kernel."""
    if "k_hist" in name or "k_partition" in name:
        return 4 * n
    if "k_bucket" in name or "k_scan" in name:
        return 4 * U
    if "k_fill" in name:
        return 4 * n + 4 * U if mode == "sort" else 0
    return 0


def source_digest(top: str = "dialsort.hip") -> str:
    """sha256 over the sources the single-array path's kernels are built from:
    `top` and every file under csrc/ it includes, transitively (names and
    contents).  The public header, which only declares the C ABI, is left out."""
    import hashlib
    import re

    d = os.path.join(ROOT, "paper_2605_16667_amd", "csrc")
    inc = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)
    seen, todo = set(), [os.path.normpath(os.path.join(d, top))]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(f) or os.path.dirname(f) != d:
            continue
        seen.add(f)
        with open(f) as fh:
            todo += [os.path.normpath(os.path.join(os.path.dirname(f), m)) for m in inc.findall(fh.read())]
    h = hashlib.sha256()
    for f in sorted(seen):
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _kname(s: str) -> str:
    return s.replace("ds::", "").replace("(", "").replace(")", "").replace(" ", "")


def profiled_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it
    was taken on the current sources: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) each times the factor that maps the same counter onto the bytes of
    a plain device copy.  None when absent or stale."""
    path = os.path.join(ROOT, "profiles", "large_uniform_sort_counters.txt")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    digest, fs, ws, vals = None, None, None, {}
    for ln in lines:
        if ln.startswith("# source-sha256:"):
            digest = ln.split(":", 1)[1].strip()
        elif ln.startswith("# scale:"):
            parts = dict(x.split("=") for x in ln.split(":", 1)[1].split())
            fs, ws = float(parts["fetch"]), float(parts["write"])
        elif not ln.startswith("#") and ln.strip():
            cols = ln.split()
            if len(cols) >= 4 and cols[-3] in ("FETCH_SIZE", "WRITE_SIZE"):
                vals[(_kname(" ".join(cols[:-3])), cols[-3])] = float(cols[-1])
    if digest != source_digest() or fs is None:
        return None
    k = _kname(kernel)
    f, w_ = vals.get((k, "FETCH_SIZE")), vals.get((k, "WRITE_SIZE"))
    if f is None or w_ is None:
        return None
    return {"bytes": (f * fs + w_ * ws) * 1024.0, "fetch_bytes": f * fs * 1024.0, "write_bytes": w_ * ws * 1024.0,
            "source": "profiles/large_uniform_sort_counters.txt"}


def time_calls(ds, hip, call, K, W, n, U, nev=12):
    """W untimed calls, then K timed calls between two events (the step time:
    the whole K steps over K), then K calls with an event at every step
    boundary (the spread of single steps), then K more calls with an event
    after every launch (the per-kernel times).  Events between steps add a
    little to each step, so the step time comes from the first pass.  Returns
    a dict."""
    import torch

    for _ in range(W):
        call()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for k in range(K):
        call()
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    marks[0].record(stream)
    for k in range(K):
        call()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    steps = [marks[k].elapsed_time(marks[k + 1]) for k in range(K)]
    evsets = [hip.make(nev) for _ in range(K)]
    count = ctypes.c_uint32(0)
    for k in range(K):
        ds.dialsort_set_launch_events(evsets[k], nev, count)
        call()
    ds.dialsort_set_launch_events(None, 0, None)
    torch.cuda.synchronize()
    nl = count.value
    names = [ds.dialsort_launch_name(i) for i in range(nl)]
    per_kernel = {}
    for i, name in enumerate(names):
        d = [hip.ms(e[i], e[i + 1]) for e in evsets]
        key = f"{i}:{name}"
        per_kernel[key] = {"avg_ms": statistics.fmean(d), "min_ms": min(d)}
    evented = [hip.ms(e[0], e[nl]) for e in evsets]
    for e in evsets:
        hip.free(e)
    ms_step = total_ms / K
    return {
        "ms_per_step": ms_step,
        "best_ms": min(steps),
        "median_ms": statistics.median(steps),
        "cv": (statistics.pstdev(steps) / statistics.fmean(steps)) if len(steps) > 1 else 0.0,
        "ms_per_step_with_step_events": statistics.fmean(steps),
        "ms_per_step_with_launch_events": statistics.fmean(evented),
        "kernels": per_kernel,
        "names": names,
    }


def roofline_of(res, n, U, mode):
    kname, kst = max(res["kernels"].items(), key=lambda kv: kv[1]["avg_ms"])
    name = kname.split(":", 1)[1]
    b = algo_bytes(name, n, U, mode)
    ach = b / (kst["avg_ms"] * 1e-3)
    tr = profiled_traffic(name)
    return {"bound": "hbm", "kernel": name, "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": ach / HBM_PEAK, "traffic": tr["bytes"] if tr else None, "avg_ms": kst["avg_ms"],
            "algo_bytes": b, "traffic_detail": tr}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bytes read plus bytes written per second by a plain device-to-device copy
    (torch's copy kernel) of nbytes: the bandwidth this GPU reaches on a pure
    stream, the practical ceiling beside the 8 TB/s peak."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3)


def with_copy_ceiling(pr, copy_bps):
    pr = dict(pr)
    pr["copy_GBps"] = copy_bps / 1e9
    pr["frac_of_copy"] = pr["achieved_GBps"] * 1e9 / copy_bps
    return pr


VERIFY_RUNS = 3  # verified runs after the timed ones


def verify_sort(keys, U, H, out):
    """Independent device-side check with torch ops: H is the bincount of the keys
    and the output is nondecreasing with the same bincount."""
    import torch

    kl = keys.to(torch.int64) & 0xFFFFFFFF
    ref = torch.bincount(kl, minlength=U)
    Hl = H.to(torch.int64) & 0xFFFFFFFF
    ok = bool(torch.equal(ref, Hl))
    del kl, ref
    if out is not None:
        ol = out.to(torch.int64) & 0xFFFFFFFF
        ok = ok and bool((ol[1:] >= ol[:-1]).all()) and bool(torch.equal(torch.bincount(ol, minlength=U), Hl))
        del ol
    return ok


def run_sort_workload(ds, hip, keys, U, K, W, mode="sort"):
    import torch

    n = keys.numel()
    dev = keys.device
    H = torch.empty(U, dtype=torch.int32, device=dev)
    if mode == "sort":
        out = torch.empty(n, dtype=torch.int32, device=dev)
        ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT), dev)
        call = lambda: ds.check(ds.dialsort_sort(keys, U, H, out, ws))  # noqa: E731
    else:
        out = None
        ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_HISTOGRAM), dev)
        call = lambda: ds.check(ds.dialsort_histogram(keys, U, H, ws))  # noqa: E731
    res = time_calls(ds, hip, call, K, W, n, U)
    st = ds.dialsort_status_sync(ws)
    if st != ds.DIALSORT_OK:
        raise RuntimeError(f"device status {st}: {ds.dialsort_strerror(st)}")
    checks = [verify_sort(keys, U, H, out)]  # the last timed run
    # then a few more runs, each from poisoned outputs and each verified
    for _ in range(VERIFY_RUNS):
        H.fill_(-1)
        if out is not None:
            out.fill_(-1)
        call()
        checks.append(ds.dialsort_status_sync(ws) == ds.DIALSORT_OK and verify_sort(keys, U, H, out))
    res["verified"] = all(checks)
    res["verified_runs"] = len(checks)
    algo = (8 * n + 8 * U) if mode == "sort" else (4 * n + 4 * U)
    res["keys_per_s"] = n / (res["ms_per_step"] * 1e-3)
    res["path_roofline"] = {"algo_bytes": algo, "achieved_GBps": algo / (res["ms_per_step"] * 1e-3) / 1e9,
                            "frac": algo / (res["ms_per_step"] * 1e-3) / HBM_PEAK}
    res["roofline"] = roofline_of(res, n, U, mode)
    del H, out, ws
    return res


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def verify_batch(arrays):
    ok = True
    for (k, U, H, o) in arrays:
        ok = ok and verify_sort(k, U, H, o)
        if not ok:
            break
    return ok


def run_batch_workload(ds, hip, count, K, W):
    """The uneven batch: `count` independent arrays (n log-uniform in
    [2^10, 2^22], U = 2^e with e uniform on 10..20, half uniform and half
    Zipf(1.1)), sorted (a) by one autotuned fused persistent launch, captured
    in a HIP graph and replayed, and (b) by the plain form, one launch sequence
    per array (dialsort_sort_each).  Per-array latency is the time from the
    submission of the batch to the completion of that array."""
    import torch

    import workloads as w

    dev = torch.device("cuda:0")
    specs = w.batch_spec(count=count)
    arrays = []
    for s in specs:
        k = gen(s.keys(GEN_DEVICE))
        arrays.append((k, s.U, torch.empty(s.U, dtype=torch.int32, device=dev),
                       torch.empty(s.n, dtype=torch.int32, device=dev)))
    torch.cuda.synchronize()
    nkeys = sum(s.n for s in specs)
    algo = sum(8 * s.n + 8 * s.U for s in specs)
    descs = ds.make_descs(arrays)
    ws = ds.workspace(ds.dialsort_batched_workspace_bytes(descs, count), dev)
    log(f"batch: {count} arrays, {nkeys} keys, workspace {ws.numel() / 2**30:.2f} GiB; autotuning")
    t0 = time.perf_counter()
    st, cfg = ds.dialsort_batch_autotune(descs, count, ws)
    ds.check(st)
    tune_s = time.perf_counter() - t0
    st, plan = ds.dialsort_batch_prepare(descs, count, cfg, ws)
    ds.check(st)
    # fused: graph of the launch, replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            ds.check(ds.dialsort_batch_launch(plan, stream=side))
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(W):
        g.replay()
    torch.cuda.synchronize()
    ev = hip.make(2 * K)
    stream = torch.cuda.current_stream()
    lib = hip.lib
    lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    times = []
    for i in range(K):
        lib.hipEventRecord(ev[2 * i], ctypes.c_void_p(stream.cuda_stream))
        g.replay()
        lib.hipEventRecord(ev[2 * i + 1], ctypes.c_void_p(stream.cuda_stream))
    torch.cuda.synchronize()
    times = [hip.ms(ev[2 * i], ev[2 * i + 1]) for i in range(K)]
    hip.free(ev)
    st = ds.dialsort_status_sync(ws)
    if st != ds.DIALSORT_OK:
        raise RuntimeError(f"device status {st}")
    st, arr_ms, launch_ms, unit_ms = ds.dialsort_batch_times(plan, count, units=True)
    ds.check(st)
    fused_ms = statistics.median(times)
    lead = max(0.0, times[-1] - launch_ms)  # submission to the first unit
    lat = [t + lead for t in arr_ms]
    fused = {"ms": fused_ms, "best_ms": min(times), "keys_per_s": nkeys / (fused_ms * 1e-3),
             "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99), "max_ms": max(lat),
             "launch_ms_device": launch_ms,
             "path_roofline": {"algo_bytes": algo, "achieved_GBps": algo / (fused_ms * 1e-3) / 1e9,
                               "frac": algo / (fused_ms * 1e-3) / HBM_PEAK},
             "config": {"block": cfg.block, "log2_width": cfg.log2_width, "chunk_keys": cfg.chunk_keys},
             "units": plan.units, "grid": plan.grid, "autotune_s": tune_s,
             "unit_wg_ms": {k: [round(v[0], 3), round(v[1], 3)] for k, v in unit_ms.items()}}
    fused["verified"] = verify_batch(arrays)
    log(f"batch fused: {fused_ms:.3f} ms, p50 {fused['p50_ms']:.3f} p99 {fused['p99_ms']:.3f} "
        f"verified={fused['verified']} cfg={fused['config']}")
    del g
    # plain: one launch sequence per array, launch events for per-array completion
    for (k, U, H, o) in arrays:
        H.fill_(-1)
        o.fill_(-1)
    ncap = 6 * count + 8
    evs = hip.make(ncap)
    cnt = ctypes.c_uint32(0)
    Kl = max(2, K // 2)
    loop_ms, loop_lat = [], None
    for it in range(1 + Kl):
        ds.check(ds.dialsort_set_launch_events(evs, ncap, cnt))
        ds.check(ds.dialsort_sort_each(descs, count, ws))
        nl = cnt.value
        names = [ds.dialsort_launch_name(i) for i in range(nl)]
        ds.check(ds.dialsort_set_launch_events(None, 0, None))
        torch.cuda.synchronize()
        if it == 0:
            continue  # warm-up
        total = hip.ms(evs[0], evs[nl])
        loop_ms.append(total)
        ends = [i + 1 for i, nm in enumerate(names) if nm and "k_or_status" in nm]
        loop_lat = [hip.ms(evs[0], evs[e]) for e in ends]
    hip.free(evs)
    st = ds.dialsort_status_sync(ws)
    if st != ds.DIALSORT_OK:
        raise RuntimeError(f"device status {st}")
    lm = statistics.median(loop_ms)
    plain = {"ms": lm, "keys_per_s": nkeys / (lm * 1e-3), "p50_ms": percentile(loop_lat, 50),
             "p99_ms": percentile(loop_lat, 99), "launches": nl,
             "path_roofline": {"algo_bytes": algo, "frac": algo / (lm * 1e-3) / HBM_PEAK}}
    plain["verified"] = verify_batch(arrays)
    log(f"batch per-array: {lm:.3f} ms, p50 {plain['p50_ms']:.3f} p99 {plain['p99_ms']:.3f} "
        f"verified={plain['verified']}")
    res = {"workload": f"{count} uneven arrays: n log-uniform in [2^10, 2^22], U = 2^e, e uniform on 10..20, "
                       "half uniform, half Zipf(1.1)", "arrays": count, "keys": nkeys,
           "fused_graph": fused, "per_array_launches": plain, "speedup": lm / fused_ms}
    del arrays, ws
    torch.cuda.empty_cache()
    return res


PROFILE_CASES = ("large-sort", "large-hist", "plain", "skewed-sort", "skewed-hist", "uniform28-sort",
                 "uniform28-hist", "batch", "zipf24-sort", "global-hist")


def run_profile_case(ds, hip, name, K, W, batch_count):
    """One workload alone (--profile NAME), for profiler runs: every dispatch of
    the process then belongs to that one input.  No autotuning, no graph and no
    per-array baseline for the batch (it launches the plan prepared with the
    configuration the autotuner picks on this batch, 1024 threads, W = 2^16,
    chunks of 2^22 keys).  Prints one JSON line with the per-kernel times."""
    import torch

    import workloads as w

    if name == "batch":
        specs = w.batch_spec(count=batch_count)
        dev = torch.device("cuda:0")
        arrays = []
        for sp in specs:
            k = gen(sp.keys(GEN_DEVICE))
            arrays.append((k, sp.U, torch.empty(sp.U, dtype=torch.int32, device=dev),
                           torch.empty(sp.n, dtype=torch.int32, device=dev)))
        descs = ds.make_descs(arrays)
        ws = ds.workspace(ds.dialsort_batched_workspace_bytes(descs, batch_count), dev)
        st, plan = ds.dialsort_batch_prepare(descs, batch_count, ds.batch_config(1024, 16, 1 << 22), ws)
        ds.check(st)
        call = lambda: ds.check(ds.dialsort_batch_launch(plan))  # noqa: E731
        res = time_calls(ds, hip, call, K, W, 0, 0)
        st = ds.dialsort_status_sync(ws)
        ok = st == ds.DIALSORT_OK and verify_batch(arrays[::64])  # a sample: every 64th array
        print(json.dumps({"profile": name, "arrays": batch_count, "ms_per_step": res["ms_per_step"],
                          "kernels": res["kernels"], "verified": ok}), flush=True)
        return
    if name.startswith("large"):
        keys, U = w.uniform(10**8, 1 << 24, w.BASE_SEED + 1, "cuda"), 1 << 24
    elif name == "plain":
        keys, U = w.uniform(1 << 20, 1 << 16, w.BASE_SEED, "cuda"), 1 << 16
    elif name.startswith("skewed"):
        keys, U = gen(w.hot_zipf(1 << 28, 1 << 16, w.BASE_SEED + 2, GEN_DEVICE)), 1 << 16
    elif name == "zipf24-sort":
        # heavy buckets split between workgroups (global atomics into scratch rows)
        keys, U = gen(w.zipf(10**8, 1 << 24, 1.2, w.BASE_SEED + 5, GEN_DEVICE)), 1 << 24
    elif name == "global-hist":
        # a universe beyond the partitioned path: direct global atomics into H
        keys, U = w.uniform(1 << 24, 1 << 30, w.BASE_SEED + 6, "cuda"), 1 << 30
    else:
        keys, U = w.uniform(1 << 28, 1 << 16, w.BASE_SEED + 2, "cuda"), 1 << 16
    torch.cuda.synchronize()
    r = run_sort_workload(ds, hip, keys, U, K, W, "hist" if name.endswith("-hist") else "sort")
    print(json.dumps({"profile": name, "n": keys.numel(), "U": U, "ms_per_step": r["ms_per_step"],
                      "kernels": r["kernels"], "verified": r["verified"]}), flush=True)


def run_serve_workload(ds, hip, num, loads, batch_cfg):
    """The served stream: `num` requests with Poisson arrivals, n log-uniform
    in [2^12, 2^24], U uniform over {2^12, 2^16, 2^20, 2^24}, uniform or
    Zipf(1.2) keys (p = 1/2), all keys already in device memory.  For every
    load L the arrival rate is L / (mean serial service time).  Baseline: serial
    plain sorts, first in first out, one dialsort_sort at a time; served: the
    continuous-batching server.  Latency = arrival to the moment the host sees
    the request complete, on the host clock for both: the serial loop after its
    synchronisation, the server when a poll first finds the request's batch
    finished (seen_ms, on the server clock, against arrivals placed on that
    clock).  Served results stay resident until the replay ends; every request's
    H and output are then checked (torch bincount and order) before release."""
    import torch

    import workloads as w

    dev = torch.device("cuda:0")
    probe = w.request_stream(num, 1.0)
    keys = [gen(r.spec.keys(GEN_DEVICE)) for r in probe]
    torch.cuda.synchronize()
    nkeys = sum(r.spec.n for r in probe)
    nmax = max(r.spec.n for r in probe)
    Umax = max(r.spec.U for r in probe)
    H = torch.empty(Umax, dtype=torch.int32, device=dev)
    out = torch.empty(nmax, dtype=torch.int32, device=dev)
    ws = ds.workspace(max(ds.dialsort_workspace_bytes(r.spec.n, r.spec.U, ds.DIALSORT_MODE_SORT) for r in probe), dev)
    # serial service times (each sort alone, warm)
    for i in range(min(8, num)):
        ds.check(ds.dialsort_sort(keys[i], probe[i].spec.U, H, out, ws))
    torch.cuda.synchronize()
    svc = []
    for k, r in zip(keys, probe):
        t = time.perf_counter()
        ds.check(ds.dialsort_sort(k, r.spec.U, H, out, ws))
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t)
    mean_svc = statistics.mean(svc)
    # every result stays resident until the replay ends: the arena holds all
    # footprints plus room for the batches' workspaces
    foot = sum(ds.dialsort_server_footprint(r.spec.n, r.spec.U) for r in probe)
    arena_bytes = foot + (16 << 30)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    res = {"workload": f"{num} requests, Poisson arrivals at L x (1 / mean serial service time), "
                       "n log-uniform in [2^12, 2^24], U in {2^12, 2^16, 2^20, 2^24}, uniform or Zipf(1.2)",
           "requests": num, "keys": nkeys, "mean_serial_service_ms": mean_svc * 1e3,
           "latency": "arrival to host-observed completion, host clock for both forms",
           "server_config": {"block": batch_cfg.block, "log2_width": batch_cfg.log2_width,
                             "chunk_keys": batch_cfg.chunk_keys, "max_inflight": SERVE_SLOTS, "max_batch": 256,
                             "arena_bytes": arena_bytes},
           "loads": {}}
    for load in loads:
        rate = load / mean_svc
        reqs = w.request_stream(num, rate)
        arrivals = [r.arrival for r in reqs]
        log(f"serve L={load}: {num} requests, {nkeys} keys, mean serial service {mean_svc * 1e3:.3f} ms, "
            f"rate {rate:.1f}/s")
        # serial FIFO replay
        lat = []
        t0 = time.perf_counter()
        for k, r, a in zip(keys, reqs, arrivals):
            while time.perf_counter() - t0 < a:
                pass
            ds.check(ds.dialsort_sort(k, r.spec.U, H, out, ws))
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0 - a) * 1e3)
        span = time.perf_counter() - t0
        st = ds.dialsort_status_sync(ws)
        if st != ds.DIALSORT_OK:
            raise RuntimeError(f"device status {st}")
        serial = {"keys_per_s": nkeys / span, "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                  "mean_ms": statistics.mean(lat), "span_s": span}
        # served replay
        st, srv = ds.dialsort_server_create(arena, ds.server_config(batch_cfg, SERVE_SLOTS, 256))
        ds.check(st)
        ids, outstanding, infos = [], [], {}

        def retire_front():
            while outstanding:
                st_, info = ds.dialsort_server_info(srv, outstanding[0])
                ds.check(st_)
                if info.state != ds.DIALSORT_REQ_DONE:
                    break
                if info.status != ds.DIALSORT_OK:
                    raise RuntimeError(f"request status {info.status}")
                infos[outstanding[0]] = (info.launch_ms, info.seen_ms, info.H, info.out)
                outstanding.pop(0)

        ok = True
        try:
            t0 = time.perf_counter()
            t0s = ds.dialsort_server_now_ms(srv)
            for k, r, a in zip(keys, reqs, arrivals):
                while time.perf_counter() - t0 < a:
                    ds.check(ds.dialsort_server_poll(srv)[0])
                    retire_front()
                st, rid = ds.dialsort_server_submit(srv, k, r.spec.U)
                ds.check(st)
                ids.append(rid)
                outstanding.append(rid)
                ds.check(ds.dialsort_server_poll(srv)[0])
            while outstanding:
                ds.check(ds.dialsort_server_poll(srv)[0])
                retire_front()
            # after the replay: every served request's H and output
            for rid, k, r in zip(ids, keys, reqs):
                _, _, hp, op = infos[rid]
                ok = ok and verify_sort(k, r.spec.U, ds.arena_view(arena, hp, r.spec.U),
                                        ds.arena_view(arena, op, r.spec.n))
                ds.check(ds.dialsort_server_release(srv, rid))
        finally:
            ds.check(ds.dialsort_server_destroy(srv))
        slat = [infos[i][1] - (t0s + a * 1e3) for i, a in zip(ids, arrivals)]
        launches = sorted(set(round(infos[i][0], 6) for i in ids))
        last_seen = max(infos[i][1] for i in ids)
        served = {"keys_per_s": nkeys / ((last_seen - t0s) * 1e-3), "p50_ms": percentile(slat, 50),
                  "p99_ms": percentile(slat, 99), "mean_ms": statistics.mean(slat),
                  "span_s": (last_seen - t0s) * 1e-3, "launches": len(launches),
                  "mean_requests_per_launch": num / max(len(launches), 1), "verified": bool(ok)}
        log(f"serve L={load}: serial p50 {serial['p50_ms']:.3f} p99 {serial['p99_ms']:.3f} ms "
            f"{serial['keys_per_s'] / 1e9:.1f} Gkeys/s; served p50 {served['p50_ms']:.3f} p99 {served['p99_ms']:.3f} ms "
            f"{served['keys_per_s'] / 1e9:.1f} Gkeys/s, {len(launches)} launches, verified={ok}")
        res["loads"][str(load)] = {"rate_per_s": rate, "serial_plain": serial, "served": served}
    del H, out, ws, arena, keys
    torch.cuda.empty_cache()
    return res


def run_query_workload(ds, keys, U, K, W, nq=1 << 20):
    """Queries on the histogram of the large workload (Sec. 3.3, the canonical
    ordered state): the running count P over U bins, then nq frequency,
    presence, range-count and select queries with seeded random arguments."""
    import torch

    dev = keys.device
    H = torch.empty(U, dtype=torch.int32, device=dev)
    ws = ds.workspace(ds.dialsort_workspace_bytes(keys.numel(), U, ds.DIALSORT_MODE_HISTOGRAM), dev)
    ds.check(ds.dialsort_histogram(keys, U, H, ws))
    P = torch.empty(U + 1, dtype=torch.int64, device=dev)
    pws = ds.workspace(ds.dialsort_prefix_workspace_bytes(U), dev)
    g = torch.Generator(device=dev)
    g.manual_seed(20260321 + 40)
    q = torch.randint(0, U, (nq,), generator=g, device=dev, dtype=torch.int32)
    a = torch.randint(0, U, (nq,), generator=g, device=dev, dtype=torch.int64)
    b = torch.clamp(a + torch.randint(0, 1 << 16, (nq,), generator=g, device=dev, dtype=torch.int64), max=U)
    r = torch.randint(0, keys.numel(), (nq,), generator=g, device=dev, dtype=torch.int64)
    o32 = torch.empty(nq, dtype=torch.int32, device=dev)
    o8 = torch.empty(nq, dtype=torch.uint8, device=dev)
    o64 = torch.empty(nq, dtype=torch.int64, device=dev)
    calls = {
        "prefix": lambda: ds.check(ds.dialsort_prefix(H, U, P, pws)),
        "frequency": lambda: ds.check(ds.dialsort_query_frequency(H, U, q, o32)),
        "presence": lambda: ds.check(ds.dialsort_query_presence(H, U, q, o8)),
        "range_count": lambda: ds.check(ds.dialsort_query_range_count(P, U, a, b, o64)),
        "select": lambda: ds.check(ds.dialsort_query_select(P, U, r, o32)),
    }
    res = {"U": U, "n": keys.numel(), "queries_per_call": nq}
    for name, call in calls.items():
        for _ in range(W):
            call()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(K):
            call()
        t1.record()
        torch.cuda.synchronize()
        us = t0.elapsed_time(t1) / K * 1e3
        entry = {"us": us}
        if name == "prefix":
            entry["GBps"] = (4 * U + 8 * (U + 1)) / (us * 1e-6) / 1e9  # H read once, P written once
        else:
            entry["queries_per_s"] = nq / (us * 1e-6)
        res[name] = entry
    # a spot check against the keys (sorted with torch on the device)
    srt = torch.sort(keys.to(torch.int64) & 0xFFFFFFFF).values
    ok = bool(torch.equal(o32[:4096].to(torch.int64) & 0xFFFFFFFF, srt[r[:4096]]))
    res["verified_select_sample"] = ok
    del H, P, pws, q, a, b, r, o32, o8, o64, srt, ws
    torch.cuda.empty_cache()
    return res


def run_radix_workload(ds, K, W, sizes=(10**7, 10**8)):
    """DialSort-Radix over the whole signed int32 range (the paper's Table
    tab:radix workload: uniform int32 keys), at each size: keys/s, verified
    against torch's sort of the same keys."""
    import torch

    res = {}
    for n in sizes:
        g = torch.Generator(device="cuda")
        g.manual_seed(20260321 + 60 + n % 1000)
        keys = torch.randint(-2**31, 2**31, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        out = torch.empty_like(keys)
        ws = ds.workspace(ds.dialsort_radix_workspace_bytes(n))
        call = lambda: ds.check(ds.dialsort_sort_radix(keys, out, ws, is_signed=True))  # noqa: E731
        for _ in range(W):
            call()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(K):
            call()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / K
        ok = bool(torch.equal(out, torch.sort(keys).values))
        # one read of the keys counts all four digits; each of the four passes
        # then reads and writes them once: 36 bytes per key in all
        res[str(n)] = {"ms": ms, "keys_per_s": n / (ms * 1e-3), "verified": ok,
                       "GBps_moved": 36 * n / (ms * 1e-3) / 1e9}
        del keys, out, ws
        torch.cuda.empty_cache()
    res["paper_context"] = {"keys_per_s": 38.2e6, "n": 10**7,
                            "what": "DS-Radix, full int32 range, CPU (Table tab:radix)"}
    return res


def _time(call, K, W):
    import torch

    for _ in range(W):
        call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K


def run_transform_workload(ds, K, W, n=10**8, U=1 << 24, pieces=10):
    """The key transforms phi (Sec. 3.4) and streaming ingestion at the large
    workload's size, beside the plain sort of the same shape: signed keys in a
    2^24 range sorted through the offset map, the key range that picks it,
    indices sorted through a lookup table phi^-1, and the same n keys ingested
    into one resident H in `pieces` pieces."""
    import torch

    import workloads as w

    res = {"n": n, "U": U}
    keys = w.uniform(n, U, w.BASE_SEED + 80, "cuda")
    H = torch.empty(U, dtype=torch.int32, device="cuda")
    out = torch.empty_like(keys)
    ws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_SORT))
    lo = -(1 << 23)
    skeys = keys + lo  # signed keys in [-2^23, 2^23)
    ms = _time(lambda: ds.check(ds.dialsort_sort_offset(skeys, lo, U, H, out, ws)), K, W)
    ok = ds.dialsort_status_sync(ws) == ds.DIALSORT_OK and bool((out[1:] >= out[:-1]).all()) and \
        torch.equal(H, torch.bincount(keys, minlength=U).to(torch.int32))
    res["offset_sort"] = {"ms": ms, "keys_per_s": n / (ms * 1e-3), "verified": bool(ok)}
    mm = torch.empty(2, dtype=torch.int32, device="cuda")
    ms = _time(lambda: ds.check(ds.dialsort_key_range(skeys, mm, True)), K, W)
    ok = [int(v) for v in mm.cpu()] == [int(skeys.min()), int(skeys.max())]
    res["key_range"] = {"ms": ms, "GBps": 4 * n / (ms * 1e-3) / 1e9, "verified": bool(ok)}
    del skeys
    lut = (torch.arange(U, dtype=torch.int64, device="cuda") * 7 + 3).to(torch.int32)  # increasing
    ms = _time(lambda: ds.check(ds.dialsort_sort_lut(keys, U, lut, H, out, ws)), K, W)
    ok = ds.dialsort_status_sync(ws) == ds.DIALSORT_OK and bool((out[1:] >= out[:-1]).all()) and \
        int(out[0]) == int(lut[int(keys.min())]) and int(out[-1]) == int(lut[int(keys.max())])
    res["lut_sort"] = {"ms": ms, "keys_per_s": n / (ms * 1e-3), "verified": bool(ok)}
    ms = _time(lambda: ds.check(ds.dialsort_sort(keys, U, H, out, ws)), K, W)
    res["plain_sort_same_shape"] = {"ms": ms, "keys_per_s": n / (ms * 1e-3)}
    del lut, out, ws
    pn = n // pieces
    aws = ds.workspace(ds.dialsort_workspace_bytes(pn, U, ds.DIALSORT_MODE_ACCUMULATE))

    def stream():
        H.zero_()
        for i in range(pieces):
            ds.check(ds.dialsort_histogram_accumulate(keys[i * pn:(i + 1) * pn], U, H, aws))

    ms = _time(stream, K, W)
    ok = ds.dialsort_status_sync(aws) == ds.DIALSORT_OK and \
        torch.equal(H, torch.bincount(keys[: pieces * pn], minlength=U).to(torch.int32))
    res["accumulate"] = {"pieces": pieces, "ms": ms, "keys_per_s": pieces * pn / (ms * 1e-3), "verified": bool(ok)}
    hws = ds.workspace(ds.dialsort_workspace_bytes(n, U, ds.DIALSORT_MODE_HISTOGRAM))
    ms = _time(lambda: ds.check(ds.dialsort_histogram(keys, U, H, hws)), K, W)
    res["histogram_same_shape"] = {"ms": ms, "keys_per_s": n / (ms * 1e-3)}
    del keys, H, aws, hws
    torch.cuda.empty_cache()
    return res


def run_windows_workload(ds, K, W, count=64, wn=1 << 20, U=1 << 16):
    """A key stream sorted in tumbling windows (count windows of wn uniform
    keys, U bins): the ingestion of each window overlaps the projection of the
    previous one on a second stream, against the same calls on one stream."""
    import torch

    import workloads as w

    keys = w.uniform(count * wn, U, w.BASE_SEED + 70, "cuda")
    H = torch.empty(2 * U, dtype=torch.int32, device="cuda")
    out = torch.empty_like(keys)
    ws = ds.workspace(ds.dialsort_windows_workspace_bytes(wn, U))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def timed(two):
        ing, proj = s1, (s2 if two else s1)
        times = []
        for it in range(W + K):
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(proj)
            ing.wait_event(e0)
            ds.check(ds.dialsort_sort_windows(keys, wn, count, U, H, out, ws, ing, proj))
            e1.record(proj)
            torch.cuda.synchronize()
            if it >= W:
                times.append(e0.elapsed_time(e1))
        ok = ds.dialsort_status_sync(ws, proj) == ds.DIALSORT_OK
        last = keys[(count - 1) * wn:]
        ok = ok and verify_sort(last, U, H[((count - 1) % 2) * U:((count - 1) % 2 + 1) * U], out[(count - 1) * wn:])
        return {"ms": statistics.median(times), "best_ms": min(times),
                "keys_per_s": count * wn / (statistics.median(times) * 1e-3), "verified": bool(ok)}

    res = {"workload": f"{count} tumbling windows of {wn} uniform keys, U = {U}",
           "one_stream": timed(False), "two_streams": timed(True)}
    res["speedup"] = res["one_stream"]["ms"] / res["two_streams"]["ms"]
    del keys, H, out, ws
    torch.cuda.empty_cache()
    return res


def cpu_model():
    import platform

    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return model


def cpu_baseline(kh, U, warmup=3, runs=7):
    """The oracle as it stands, on this host, on the same keys (sequential C,
    one thread): the paper's protocol (Sec. 8.1) -- `warmup` untimed runs, then
    `runs` timed ones; best (the value), median and coefficient of variation."""
    import oracle

    n = kh.size
    times = []
    for i in range(warmup + runs):
        t = time.perf_counter()
        st, H, out = oracle.sort(kh, U)
        dt = time.perf_counter() - t
        assert st == oracle.OK
        if i >= warmup:
            times.append(dt)
    best, med = min(times), statistics.median(times)
    cv = statistics.pstdev(times) / statistics.mean(times)
    return {"value": n / best, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle.sort on the full workload (n={n}, U={U}): {warmup} warmups, best of {runs}",
            "best_s": best, "median_s": med, "cv": cv, "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def cpu_parallel_baseline(kh, U, warmup=3, runs=7):
    """The CPU-parallel baseline (private per-thread histograms, merge, projection
    by bin ranges) on all the host threads this process may use, on the same
    keys: best, median and CV of `runs` after `warmup` (Sec. 8.1's protocol),
    verified against the GPU-independent oracle's histogram."""
    import numpy as np

    import oracle
    from oracle import cpu_parallel

    T = cpu_parallel.default_threads()
    times = []
    for i in range(warmup + runs):
        t = time.perf_counter()
        st, H, out = cpu_parallel.sort(kh, U, T)
        dt = time.perf_counter() - t
        assert st == 0
        if i >= warmup:
            times.append(dt)
    st, H_ref = oracle.histogram(kh, U)
    ok = bool(st == oracle.OK and np.array_equal(H, H_ref) and out.size == kh.size
              and bool(np.all(out[1:] >= out[:-1])))
    best = min(times)
    return {"value": kh.size / best, "unit": "keys/s", "cores": T, "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "kind": "cpu-parallel baseline (oracle/cpu_parallel.c)", "best_s": best,
            "median_s": statistics.median(times), "cv": statistics.pstdev(times) / statistics.mean(times),
            "warmup": warmup, "runs": runs, "verified": ok,
            "sample": f"full workload (n={kh.size}, U={U}), histogram and sorted output"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workloads", default="large,hist,query,plain,skewed,transforms,windows,radix,batch,serve")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9,1.2",
                    help="arrival rates, as multiples of 1 / (mean serial service time)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", choices=PROFILE_CASES,
                    help="run this one workload alone (for profiler runs) instead of the benchmark")
    ap.add_argument("--host-inputs", action="store_true",
                    help="generate the Zipf and hot-key inputs on the host and copy them to the GPU")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for profiler byte counters)")
    args = ap.parse_args()
    if args.host_inputs:
        global GEN_DEVICE
        GEN_DEVICE = "cpu"
    if args.gpus != 1:
        print("bench.py measures the single-GPU hot path and runs on one GPU only; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2605_16667_amd as ds
    import workloads as w

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    hip = HipEvents()
    K, W = args.steps, args.warmup
    todo = set(args.workloads.split(","))
    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.profile:
        run_profile_case(ds, hip, args.profile, K, W, args.batch_count)
        return
    extra = {}

    copy_bps = copy_bandwidth()
    log(f"device copy: {copy_bps / 1e9:.0f} GB/s (read + write)")
    n, U = 10**8, 1 << 24
    log(f"large: generating n={n} U={U}")
    keys = w.uniform(n, U, w.BASE_SEED + 1, "cuda")
    torch.cuda.synchronize()
    log("large: sort")
    main_res = run_sort_workload(ds, hip, keys, U, K, W, "sort")
    main_res["path_roofline"] = with_copy_ceiling(main_res["path_roofline"], copy_bps)
    log(f"large: {main_res['ms_per_step']:.4f} ms/step verified={main_res['verified']}")
    if "hist" in todo:
        log("large: histogram-only")
        r = run_sort_workload(ds, hip, keys, U, K, W, "hist")
        r["path_roofline"] = with_copy_ceiling(r["path_roofline"], copy_bps)
        extra["histogram_only"] = {k: r[k] for k in ("ms_per_step", "best_ms", "median_ms", "cv", "keys_per_s",
                                                     "path_roofline", "roofline", "verified", "kernels")}
    if "query" in todo:
        log("queries on the large workload's histogram")
        extra["queries"] = run_query_workload(ds, keys, U, max(K // 2, 5), 2)
    cpu = cpu_par = None
    if not args.no_cpu:
        kh = w.as_u32(keys)
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(kh, U)
        log("cpu-parallel baseline")
        cpu_par = cpu_parallel_baseline(kh, U)
        log(f"cpu-parallel: {cpu_par['value'] / 1e6:.0f} M keys/s on {cpu_par['cores']} threads")
        del kh
    del keys
    torch.cuda.empty_cache()

    if "plain" in todo:
        n1, U1 = 1 << 20, 1 << 16
        log("plain: n=2^20 U=2^16")
        k1 = w.uniform(n1, U1, w.BASE_SEED, "cuda")
        r = run_sort_workload(ds, hip, k1, U1, max(K, 50), W, "sort")
        extra["plain"] = {"n": n1, "U": U1, "us_per_sort": r["ms_per_step"] * 1e3,
                          "best_us_with_step_events": r["best_ms"] * 1e3,
                          "us_per_sort_with_step_events": r["ms_per_step_with_step_events"] * 1e3,
                          "keys_per_s": r["keys_per_s"], "path_roofline": r["path_roofline"],
                          "verified": r["verified"], "kernels": r["kernels"]}
        del k1
    if "skewed" in todo:
        n3, U3 = 1 << 28, 1 << 16
        log("skewed: generating n=2^28 hot+Zipf(1.2)")
        k3 = gen(w.hot_zipf(n3, U3, w.BASE_SEED + 2, GEN_DEVICE))
        r = run_sort_workload(ds, hip, k3, U3, max(K // 2, 3), W, "sort")
        extra["skewed"] = {"n": n3, "U": U3, "ms_per_step": r["ms_per_step"], "keys_per_s": r["keys_per_s"],
                           "path_roofline": r["path_roofline"], "roofline": r["roofline"], "cv": r["cv"],
                           "verified": r["verified"], "kernels": r["kernels"]}
        # ingestion alone, the part the paper's skew claim is about
        r = run_sort_workload(ds, hip, k3, U3, max(K // 2, 3), W, "hist")
        extra["skewed"]["histogram_only"] = {"ms_per_step": r["ms_per_step"], "keys_per_s": r["keys_per_s"],
                                             "verified": r["verified"], "kernels": r["kernels"]}
        del k3
        torch.cuda.empty_cache()
        log("skewed: same size, uniform keys")
        k3u = w.uniform(n3, U3, w.BASE_SEED + 2, "cuda")
        r = run_sort_workload(ds, hip, k3u, U3, max(K // 2, 3), W, "sort")
        extra["uniform_same_size"] = {"n": n3, "U": U3, "ms_per_step": r["ms_per_step"],
                                      "keys_per_s": r["keys_per_s"], "path_roofline": r["path_roofline"],
                                      "verified": r["verified"], "kernels": r["kernels"]}
        extra["skew_over_uniform"] = extra["skewed"]["keys_per_s"] / r["keys_per_s"]
        r = run_sort_workload(ds, hip, k3u, U3, max(K // 2, 3), W, "hist")
        extra["uniform_same_size"]["histogram_only"] = {"ms_per_step": r["ms_per_step"],
                                                        "keys_per_s": r["keys_per_s"], "verified": r["verified"],
                                                        "kernels": r["kernels"]}
        extra["skew_over_uniform_histogram_only"] = (extra["skewed"]["histogram_only"]["keys_per_s"]
                                                     / r["keys_per_s"])
        del k3u
        torch.cuda.empty_cache()

    if "transforms" in todo:
        log("transforms: offset, key range, lookup table, accumulation at n=1e8, U=2^24")
        extra["transforms"] = run_transform_workload(ds, max(K // 2, 5), 2)
    if "windows" in todo:
        log("windows: tumbling windows, ingestion overlapped with projection")
        extra["windows"] = run_windows_workload(ds, max(K // 2, 5), 2)
        log(f"windows: one stream {extra['windows']['one_stream']['ms']:.3f} ms, "
            f"two streams {extra['windows']['two_streams']['ms']:.3f} ms")
    if "radix" in todo:
        log("radix: whole signed int32 range")
        extra["radix"] = run_radix_workload(ds, max(K // 2, 5), 2)
    batch_cfg = None
    if "batch" in todo:
        extra["batched"] = run_batch_workload(ds, hip, args.batch_count, max(K // 4, 3), 2)
        c = extra["batched"]["fused_graph"]["config"]
        batch_cfg = ds.batch_config(c["block"], c["log2_width"], c["chunk_keys"])
    if "serve" in todo:
        if batch_cfg is None:
            batch_cfg = ds.batch_config(1024, 16, 1 << 20)
        loads = [float(x) for x in args.serve_loads.split(",")]
        extra["served"] = run_serve_workload(ds, hip, args.serve_requests, loads, batch_cfg)

    line = {
        "metric": METRIC,
        "value": main_res["keys_per_s"],
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "large uniform single sort, full reconstruction", "n": n, "U": U,
                   "keys": "uniform i.i.d. on [0, 2^24)", "mode": "sort"},
        "roofline": main_res["roofline"],
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_par,
        "path_roofline": main_res["path_roofline"],
        "stats": {"best_ms": main_res["best_ms"], "median_ms": main_res["median_ms"], "cv": main_res["cv"]},
        "verified": main_res["verified"],
        "kernels": main_res["kernels"],
        "paper_context": {"value": 115.9e6, "unit": "keys/s",
                          "what": "DS-Parallel, skewed, N=1e7, U<=65536, 8-thread Intel x86-64 (CPU)"},
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
