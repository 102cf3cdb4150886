#!/usr/bin/env python3
"""Benchmark of the cumulant hot path on one MI355X.

A step is one call of cum_cumulants on resident device data: FP64 centring,
the block moment contraction of every order 2..d_max, the fixed-order FP64
chunk reduction and the cumulant recursion.  ``value`` is the effective
throughput of the mixed-precision path,
    algorithmic FLOP = sum_{d=2}^{d_max} 2 * t * stored_d
(one multiply-add per stored block entry per sample, the work of the block
method) divided by the measured step time.  The contraction itself may sum
fewer entries (with inner block size 1, each distinct sorted variable tuple
once); the roofline of the moment kernel counts the entries it does sum.
The FP64 path and any further precisions are timed on the same data and
reported beside it, each with its per-order relative error against the FP64
CPU oracle's values at sampled entries (stored in
tests/golden/bench_expected.json by tests/golden/bench_expected.py; the
benchmark runs the oracle itself only for its CPU baseline).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cumulants d=4..6: eff. TFLOP/s + MFMA util, FP64 vs mixed at stated rel error"
# MI355X dense matrix-core peaks, TFLOP/s
PEAK = {"f64": 78.6, "f32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0, "f16x2": 2500.0}
# matrix-core products issued per algorithmic multiply-add
PRODUCTS = {"f64": 1, "f32": 1, "bf16x2": 4, "bf16x3": 6, "f16x2": 3}
DTYPE = {"f64": "f64", "f32": "f32", "bf16x2": "bf16x2(f32 acc)", "bf16x3": "bf16x3(f32 acc)", "f16x2": "f16x2(f32 acc)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_flops(pc, t, n, d_max, b):
    return sum(2.0 * t * pc.layout(n, d, b)["elems"] for d in range(2, d_max + 1))


HBM_PEAK_GBS = 8000.0


def finalisation_record(pc, kinds, steps, t, n, d_max, b, prec):
    """The chunk sum and the finalisation (M = S/t and the recursion): HBM
    bound.  Algorithmic bytes per step: the chunk sum reads every chunk's sums
    and writes one (when there is more than one chunk); the finalisation reads
    one sum and writes one cumulant per stored entry."""
    info = pc.plan_info(t, n, d_max, b, prec)
    nbytes = 16.0 * info["stored_entries"]
    if info["nchunks"] > 1:
        nbytes += 8.0 * (info["nchunks"] + 1) * info["partial_entries"]
    ms = kinds["reduce"][0] / steps
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None
    return {"ms_per_step": ms, "bytes_per_step": nbytes, "GB/s": gbs,
            "frac_of_hbm": gbs / HBM_PEAK_GBS if gbs else None, "plan": info}


def time_path(torch, pc, Xd, d_max, b, prec, steps, warmup, tune):
    t, n = Xd.shape
    tuned = pc.autotune(Xd, d_max, b, prec) if tune else None
    out = {d: torch.empty(pc.layout(n, d, b)["elems"], dtype=torch.float64, device="cuda")
           for d in range(2, d_max + 1)}
    ws = torch.empty(pc.workspace_size(t, n, d_max, b, prec), dtype=torch.uint8, device="cuda")
    for _ in range(warmup):
        pc.cumulants(Xd, d_max, b, prec, ws=ws, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pc.cumulants(Xd, d_max, b, prec, ws=ws, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # second pass: the same calls with every launch bracketed by HIP events
    pc.timing_enable(True)
    pc.timing_read()
    for _ in range(steps):
        pc.cumulants(Xd, d_max, b, prec, ws=ws, out=out)
    kinds = pc.timing_read()
    pc.timing_enable(False)
    torch.cuda.synchronize()
    # third pass: one pair of events around each step, for the spread
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evs:
        e0.record()
        pc.cumulants(Xd, d_max, b, prec, ws=ws, out=out)
        e1.record()
    torch.cuda.synchronize()
    per_step = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    pct = {f"p{q}": float(np.percentile(per_step, q)) for q in (10, 50, 90)}
    return wall, kinds, out, tuned, pct


EXPECTED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "bench_expected.json")
_expected_cache = {}


def expected_case(name, t):
    """The oracle's stored values for a workload (tests/golden/bench_expected.py
    wrote them), or None if the file holds no such case with t samples."""
    if "cases" not in _expected_cache:
        try:
            with open(EXPECTED) as f:
                _expected_cache["cases"] = json.load(f)["cases"]
        except (OSError, ValueError, KeyError):
            _expected_cache["cases"] = {}
    rec = _expected_cache["cases"].get(name)
    return rec if rec is not None and rec["t"] == t else None


def stored_errors(case, kappa, other=None):
    """e_d = max |gpu - oracle| / max |oracle| over the stored sampled entries
    of each order (random positions, every pure-diagonal entry, and copies in
    blocks with a repeated block index).  With ``other`` (a dict), also the
    same maximum error over max |M_d| (the central moment at those entries),
    and the largest element-wise relative error over the entries with
    |kappa_d| >= 1e-3 max."""
    errs = {}
    for ds, o in case["orders"].items():
        d = int(ds)
        offs = np.array(o["offsets"], dtype=np.int64)
        want = np.array(o["kappa"])
        got = {p: k[d][offs] for p, k in kappa.items() if d in k}
        den = np.abs(want).max()
        errs[d] = {p: float(np.abs(g - want).max() / den) for p, g in got.items()}
        if other is not None:
            mden = np.abs(np.array(o["moment"])).max()
            big = np.abs(want) >= 1e-3 * den
            other[d] = {p: {"vs_moment": float(np.abs(g - want).max() / mden),
                            "elementwise": float((np.abs(g - want)[big] / np.abs(want)[big]).max())}
                        for p, g in got.items()}
    return errs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_rate(orc, X, n, d_max, b, pc, target_s):
    """Oracle on the first ts samples, ts sized for about target_s seconds."""
    ts = 64
    t0 = time.perf_counter()
    orc.cumulants_dense(X[:ts], d_max)
    dt = time.perf_counter() - t0
    ts = int(min(len(X), max(64, ts * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    orc.cumulants_dense(X[:ts], d_max)
    dt = time.perf_counter() - t0
    return alg_flops(pc, ts, n, d_max, b) / dt / 1e12, ts, dt


def cpu_baseline(orc, X, n, d_max, b, pc, target_s):
    """The FP64 oracle (dense over all n^d entries) on a leading slice of the
    samples, with every host thread and with one; in the benchmark's unit."""
    cores = orc.max_threads()
    value, ts, dt = _oracle_rate(orc, X, n, d_max, b, pc, target_s)
    orc.set_threads(1)
    try:
        v1, ts1, dt1 = _oracle_rate(orc, X, n, d_max, b, pc, target_s / 3)
    finally:
        orc.set_threads(cores)
    return {"value": value, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"first {ts} of {len(X)} samples, dense FP64 oracle over all n^d entries of orders 2..{d_max}, "
                      f"{dt:.1f} s; effective FLOP counted as for the GPU (2 t sum_d stored_d)",
            "seconds": dt, "cpu_model": cpu_model(),
            "single_thread": {"value": v1, "sample": f"first {ts1} samples, {dt1:.1f} s"}}


def _oracle_seconds(orc, X, d_max):
    t0 = time.perf_counter()
    orc.cumulants_dense(X, d_max)
    return time.perf_counter() - t0


def _oracle_extrapolated(orc, pc, X, n, d_max, b, n_sub, slices):
    """Dense oracle time of the full workload, extrapolated: the oracle on the
    first n_sub variables and two leading sample slices gives a + c * ts
    (a: the sample-independent recursion, c: the moment sums per sample);
    the full time is (a + c * t) * (n / n_sub)^d_max (the top order's n^d
    entries dominate both parts)."""
    t = len(X)
    # best of two runs per slice; the slices are far enough apart that the
    # per-sample part stands out of the timing noise
    times = [min(_oracle_seconds(orc, X[:ts, :n_sub], d_max) for _ in range(2)) for ts in slices]
    c = max(times[1] - times[0], 0.0) / (slices[1] - slices[0])
    a = max(times[0] - c * slices[0], 0.0)
    full = (a + c * t) * (n / n_sub) ** d_max
    return {"mode": "extrapolated",
            "sample": f"dense oracle on the first {n_sub} of {n} variables and the first {slices[0]} and "
                      f"{slices[1]} samples ({times[0]:.1f} s, {times[1]:.1f} s); full time (a + c t) "
                      f"(n / {n_sub})^{d_max}",
            "measured_seconds": times, "seconds_full": full,
            "tflops": alg_flops(pc, t, n, d_max, b) / full / 1e12}


def cpu_oracle_configs(orc, pc):
    """The dense FP64 oracle (every n^d entry, all host threads) on the other
    workloads, as a stated CPU baseline: the n = 16 workload in full, the
    first 16 datasets of the 512-dataset batch in full, and the n = 24 (d <= 6)
    and n = 64 (d <= 5) workloads extrapolated from timed slices."""
    import workloads

    out = {"cores": orc.max_threads(), "cpu_model": cpu_model()}
    name = "t-wishart-n16-t5000"
    w = workloads.WORKLOADS[name]
    X = workloads.generate(name)
    dt = _oracle_seconds(orc, X, w["d_max"])
    cores = orc.max_threads()
    orc.set_threads(1)
    try:
        dt1 = _oracle_seconds(orc, X, w["d_max"])
    finally:
        orc.set_threads(cores)
    fl = alg_flops(pc, w["t"], w["n"], w["d_max"], w["b"])
    out[name] = {"mode": "full dense", "seconds": dt, "tflops": fl / dt / 1e12,
                 "single_thread": {"seconds": dt1, "tflops": fl / dt1 / 1e12}}
    log(f"  oracle {name}: {dt:.2f} s ({dt1:.2f} s on one thread)")
    name = "batch512-t-corr-n32"
    w = workloads.WORKLOADS[name]
    Xs = workloads.generate(name)[:16]
    dt = sum(_oracle_seconds(orc, X, w["d_max"]) for X in Xs)
    fl = sum(alg_flops(pc, len(X), w["n"], w["d_max"], w["b"]) for X in Xs)
    out[name] = {"mode": "full dense on the first 16 of the 512 datasets", "seconds": dt,
                 "datasets_per_s": 16 / dt, "tflops": fl / dt / 1e12,
                 "samples": int(sum(len(X) for X in Xs))}
    log(f"  oracle {name} (16 datasets): {dt:.2f} s")
    for name, n_sub, slices in [("laplace-mix-n24-t200000", 16, (32, 512)), ("ar1-garch-n64-t50000", 32, (64, 448))]:
        w = workloads.WORKLOADS[name]
        X = workloads.generate(name)
        out[name] = _oracle_extrapolated(orc, pc, X, w["n"], w["d_max"], w["b"], n_sub, slices)
        log(f"  oracle {name}: {out[name]['seconds_full']:.0f} s extrapolated")
    return out


def bench_batched(torch, pc, prec, steps, warmup, tune, per_dataset=True):
    """The 512-dataset workload: one graph replay per step vs one
    cum_cumulants call per dataset (unless per_dataset is false); datasets/s
    and per-dataset latency."""
    import workloads

    name = "batch512-t-corr-n32"
    w = workloads.WORKLOADS[name]
    n, b, d_max = w["n"], w["b"], w["d_max"]
    Xs = workloads.generate(name)
    ts = [len(X) for X in Xs]
    Xd = [torch.from_numpy(X).cuda() for X in Xs]
    flops = sum(alg_flops(pc, t, n, d_max, b) for t in ts)
    uflops = sum(alg_flops(pc, t, n, d_max, 1) for t in ts)
    batch = pc.Batch(ts, n, d_max, b, prec)
    tuned = batch.autotune(Xd) if tune else None
    out = [{d: torch.empty(pc.layout(n, d, b)["elems"], dtype=torch.float64, device="cuda")
            for d in range(2, d_max + 1)} for _ in ts]
    means = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in ts]
    for _ in range(warmup):
        batch.run(Xd, out=out, means=means)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run(Xd, out=out, means=means)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    start, ticks, hz = batch.timestamps()
    lat = np.array([(tk - start) / hz * 1e3 for tk in ticks])
    batch.close()
    rec = {"workload": name, "n_sets": len(ts), "prec": prec, "t_total": int(sum(ts)),
           "ms_per_batch": ms, "datasets_per_s": len(ts) / ms * 1e3, "eff_tflops": flops / (ms * 1e-3) / 1e12,
           "tflops_unique": uflops / (ms * 1e-3) / 1e12,
           "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
           "tuning": tuned}
    if not per_dataset:
        return rec
    # one launch sequence per dataset, same precision, buffers preallocated
    wsz = max(pc.workspace_size(t, n, d_max, b, prec) for t in ts)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    for s in range(min(8, len(ts))):
        pc.cumulants(Xd[s], d_max, b, prec, ws=ws, out=out[s])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in ts]
    t0 = time.perf_counter()
    ev0.record()
    for s in range(len(ts)):
        pc.cumulants(Xd[s], d_max, b, prec, ws=ws, out=out[s])
        evs[s].record()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    seq_lat = np.array([ev0.elapsed_time(e) for e in evs])
    rec["per_dataset_calls"] = {"ms_total": seq_ms, "datasets_per_s": len(ts) / seq_ms * 1e3,
                                "latency_ms_p50": float(np.percentile(seq_lat, 50)),
                                "latency_ms_p99": float(np.percentile(seq_lat, 99))}
    return rec


def bench_workloads(torch, pc, steps, tune):
    """The higher-order workloads (d_max = 6 and 5) in every precision (FP32,
    FP64, the two- and three-term BF16 splits and the FP16 split): step time, effective
    throughput (the block method's FLOP, 2 t sum_d stored_d) and the same
    time against the distinct-tuple lower bound (2 t sum_d C(n+d-1, d)),
    moment-kernel throughput and matrix-unit fraction (issued products:
    4 or 6 per FMA for the BF16 splits, 3 for the FP16 split), and e_d per order against the
    oracle's stored values at about 300 sampled entries per order (random
    positions, every pure diagonal, and copies in blocks with repeated block
    indices)."""
    import workloads

    out = {}
    for name in ["laplace-mix-n24-t200000", "ar1-garch-n64-t50000"]:
        w = workloads.WORKLOADS[name]
        n, b, d_max, t = w["n"], w["b"], w["d_max"], w["t"]
        log(f"workload {name}")
        X = workloads.generate(name)
        Xd = torch.from_numpy(X).cuda()
        flops = alg_flops(pc, t, n, d_max, b)
        uflops = alg_flops(pc, t, n, d_max, 1)
        res, kap = {}, {}
        for p in ["f32", "f64", "bf16x3", "bf16x2", "f16x2"]:
            wall, kinds, o, tuned, pct = time_path(torch, pc, Xd, d_max, b, p, steps, 2, tune)
            cfg = pc.get_tuning(t, n, d_max, b, p)
            kflops = alg_flops(pc, t, n, d_max, cfg["inner_b"])
            per_launch = kinds["moment"][0] / max(kinds["moment"][1], 1)
            mt = kflops / (per_launch * 1e-3) / 1e12
            res[p] = {"ms_per_step": wall * 1e3, "tflops": flops / wall / 1e12,
                      "tflops_unique": uflops / wall / 1e12, "ms_per_step_pct": pct,
                      "moment_ms_per_launch": per_launch, "moment_tflops": mt,
                      "mfma_frac": mt * PRODUCTS[p] / PEAK[p], "config": cfg,
                      "kernel_ms": {k: v[0] / steps for k, v in kinds.items() if v[1]},
                      "finalisation": finalisation_record(pc, kinds, steps, t, n, d_max, b, p)}
            kap[p] = {d: o[d].cpu().numpy() for d in o}
            log(f"  {p}: {wall * 1e3:.3f} ms/step, {flops / wall / 1e12:.2f} eff TFLOP/s "
                f"({uflops / wall / 1e12:.2f} on distinct tuples); moment kernel {mt:.1f} TFLOP/s")
        case = expected_case(name, t)
        errs = stored_errors(case, kap) if case else {}
        for p in res:
            res[p]["rel_err"] = {str(d): errs[d][p] for d in errs}
            log(f"  {p}: e_d " + " ".join(f"{d}:{errs[d][p]:.2e}" for d in errs))
        out[name] = {"n": n, "b": b, "d_max": d_max, "t": t, "alg_flop_per_step": flops,
                     "unique_flop_per_step": uflops, "paths": res}
    return out


def bench_high_orders(torch, pc, steps):
    """Orders to 8 and 10 (the recursion's partition tables grow to 715 and
    17722 terms per entry): step time, effective throughput, the split of
    kernel time between the contraction and the finalisation, and e_d of the
    top orders against the oracle's stored values (FP32 requested,
    autotuned like the other workloads; from d_max = 7 on the library stages
    and contracts in FP64, since FP32-rounded samples alone put e_8 above
    1e-6)."""
    import workloads

    out = {}
    for n, b, d_max, t in [(16, 2, 8, 20_000), (8, 2, 10, 20_000)]:
        name = f"laplace-mix-n{n}-t{t}-d{d_max}"
        log(f"high orders {name}")
        X = workloads.laplace_mix(t=t, n=n, seed=1701006)
        Xd = torch.from_numpy(X).cuda()
        flops = alg_flops(pc, t, n, d_max, b)
        wall, kinds, o, tuned, pct = time_path(torch, pc, Xd, d_max, b, "f32", steps, 2, True)
        ms = {k: v[0] / steps for k, v in kinds.items() if v[1]}
        case = expected_case(name, t)
        kap = {"f32": {d: o[d].cpu().numpy() for d in (d_max - 1, d_max)}}
        errs = {str(d): e["f32"] for d, e in stored_errors(case, kap).items()} if case else {}
        uflops = alg_flops(pc, t, n, d_max, 1)
        out[name] = {"n": n, "b": b, "d_max": d_max, "t": t, "prec": "f32", "contraction_prec": "f64", "ms_per_step": wall * 1e3,
                     "ms_per_step_pct": pct, "tflops": flops / wall / 1e12,
                     "tflops_unique": uflops / wall / 1e12, "kernel_ms": ms,
                     "stored_entries": pc.plan_info(t, n, d_max, b, "f32")["stored_entries"],
                     "tuned": tuned, "rel_err_sampled": errs}
        log(f"  {wall * 1e3:.3f} ms/step, {flops / wall / 1e12:.2f} eff TFLOP/s; kernels {ms}; e {errs}")
    return out


def bench_small(torch, pc, steps, tune):
    """The launch-bound workload (n = 16, t = 5000, d <= 4, b = 2, FP64 path):
    per-call latency of eager calls and of replays of a HIP graph captured
    from one call (autotuned like the other paths)."""
    import workloads

    name = "t-wishart-n16-t5000"
    w = workloads.WORKLOADS[name]
    n, b, d_max, t = w["n"], w["b"], w["d_max"], w["t"]
    Xd = torch.from_numpy(workloads.generate(name)).cuda()
    tuned = pc.autotune(Xd, d_max, b, "f64") if tune else None
    out = {d: torch.empty(pc.layout(n, d, b)["elems"], dtype=torch.float64, device="cuda")
           for d in range(2, d_max + 1)}
    ws = torch.empty(pc.workspace_size(t, n, d_max, b, "f64"), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        pc.cumulants(Xd, d_max, b, "f64", ws=ws, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pc.cumulants(Xd, d_max, b, "f64", ws=ws, out=out)
    e1.record()
    torch.cuda.synchronize()
    eager_us = e0.elapsed_time(e1) / steps * 1e3
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            pc.cumulants(Xd, d_max, b, "f64", ws=ws, out=out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_us = e0.elapsed_time(e1) / steps * 1e3
    flops = alg_flops(pc, t, n, d_max, b)
    return {"workload": name, "prec": "f64", "eager_us_per_call": eager_us, "graph_us_per_replay": graph_us,
            "eff_tflops_graph": flops / (graph_us * 1e-6) / 1e12, "tuning": tuned}


def bench_streaming(torch, pc, X, n, d_max, b, prec, steps, batch=10_000, window=5):
    """A rolling window over the benchmark data: `window` batches of `batch`
    samples; one slide adds the next batch and removes the oldest (two
    updates).  Reports the slide time, the update rate (samples and FLOP: the
    contraction of each update sums every sorted variable tuple of orders
    2..d_max once), the latency of the window's cumulants by the recursion and
    by the general formula, and both against one FP64 call on the window's
    samples."""
    t = X.shape[0]
    nb = t // batch
    Xd = torch.from_numpy(X).cuda()
    batches = [Xd[i * batch:(i + 1) * batch] for i in range(nb)]
    st = pc.Stream(n, d_max, b, prec)
    try:
        for i in range(window):
            st.add(batches[i])
        first = 0

        def slide(k):
            st.add(batches[(first + window + k) % nb])
            st.remove(batches[(first + k) % nb])

        for k in range(2):
            slide(k)
        first += 2
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            slide(k)
        e1.record()
        torch.cuda.synchronize()
        first += steps
        slide_ms = e0.elapsed_time(e1) / steps
        lat, res = {}, {}
        for method in ("recursion", "moebius"):
            st.cumulants(method=method)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(5):
                mean, K = st.cumulants(method=method)
            e1.record()
            torch.cuda.synchronize()
            lat[method] = e0.elapsed_time(e1) / 5
            res[method] = {d: K[d].cpu().numpy() for d in K}
        win = torch.cat([batches[(first + i) % nb] for i in range(window)])
        _, R = pc.cumulants(win, d_max, b, "f64")
        ref = {d: R[d].cpu().numpy() for d in R}
    finally:
        st.close()
    diff = {m: {str(d): float(np.abs(res[m][d] - ref[d]).max() / np.abs(ref[d]).max()) for d in ref} for m in res}
    uflop = 2.0 * batch * sum(math.comb(n + d - 1, d) for d in range(2, d_max + 1))
    return {"workload": f"rolling window of {window} x {batch} samples over the benchmark data", "prec": prec,
            "batch": batch, "window_batches": window, "ms_per_slide": slide_ms,
            "samples_per_s": 2 * batch / (slide_ms * 1e-3),
            "update_tflops": 2 * uflop / (slide_ms * 1e-3) / 1e12,
            "cumulants_ms": lat, "rel_diff_vs_one_call_f64": diff}


def profile_record(prec, workload):
    """The committed rocprofv3 counter summary of the moment kernel (HBM bytes
    and matrix-unit use per launch), if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", f"moment_kernel_{prec}_{workload}.pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1701_05420_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernels_hip_sha256") != sha:
        return None
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="t-gamma-mix-n48-t100000")
    ap.add_argument("--prec", default="f32", help="precision of the reported path")
    ap.add_argument("--compare", default="f64,bf16x3,bf16x2,f16x2", help="further precisions timed on the same data")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (planner defaults)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-dataset batched measurement")
    ap.add_argument("--no-workloads", action="store_true", help="skip the d_max = 5, 6 workloads")
    ap.add_argument("--no-streaming", action="store_true", help="skip the rolling-window measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (to scale HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        nbytes = 512 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 10}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X (sharding across GPUs "
              "is not built); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1701_05420_amd as pc
    import workloads

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = workloads.WORKLOADS[args.workload]
    if w["t"] is None:
        print("the batched workload is measured by --workload of a single dataset; see tests", file=sys.stderr)
        sys.exit(2)
    n, b, d_max, t = w["n"], w["b"], w["d_max"], w["t"]
    log(f"workload {args.workload}: n={n} b={b} d_max={d_max} t={t}")
    X = workloads.generate(args.workload)
    Xd = torch.from_numpy(X).cuda()
    flops = alg_flops(pc, t, n, d_max, b)
    uflops = alg_flops(pc, t, n, d_max, 1)  # each distinct sorted variable tuple once

    precs = [args.prec] + [p for p in args.compare.split(",") if p and p != args.prec]
    res, kappa = {}, {}
    for p in precs:
        log(f"timing {p}")
        wall, kinds, out, tuned, pct = time_path(torch, pc, Xd, d_max, b, p, args.steps, args.warmup,
                                                 not args.no_tune)
        mom_ms, mom_n = kinds["moment"]
        per_launch = mom_ms / max(mom_n, 1)
        cfg = pc.get_tuning(t, n, d_max, b, p)
        kflops = alg_flops(pc, t, n, d_max, cfg["inner_b"])  # entries the contraction sums
        achieved = kflops / (per_launch * 1e-3) / 1e12
        res[p] = {"ms_per_step": wall * 1e3, "tflops": flops / wall / 1e12, "ms_per_step_pct": pct,
                  "tflops_unique": uflops / wall / 1e12,
                  "moment_ms_per_launch": per_launch, "moment_tflops": achieved,
                  "moment_flop_per_launch": kflops,
                  "mfma_frac": achieved * PRODUCTS[p] / PEAK[p],
                  "kernel_ms": {k: v[0] / args.steps for k, v in kinds.items() if v[1]},
                  "finalisation": finalisation_record(pc, kinds, args.steps, t, n, d_max, b, p),
                  "tuning": tuned, "config": cfg}
        kappa[p] = {d: out[d].cpu().numpy() for d in out}
        log(f"  {p}: {wall * 1e3:.3f} ms/step, {flops / wall / 1e12:.2f} eff TFLOP/s; "
            f"moment kernel {per_launch:.3f} ms = {achieved:.2f} TFLOP/s")

    errs_other = {}
    case = None if args.no_errors else expected_case(args.workload, t)
    errs = stored_errors(case, kappa, other=errs_other) if case else {}
    main_p = args.prec
    r = res[main_p]
    prof = profile_record(main_p, args.workload)
    prof_alg = r["moment_flop_per_launch"] * PRODUCTS[main_p]
    roof = {"bound": "mfma", "achieved": r["moment_tflops"] * PRODUCTS[main_p], "peak": PEAK[main_p],
            "unit": "TFLOP/s", "frac": r["moment_tflops"] * PRODUCTS[main_p] / PEAK[main_p],
            "traffic": prof.get("hbm_bytes_per_launch") if prof else None,
            "mfma_util_pmc": ({"issued_frac_of_peak": prof["mfma_issued_frac_of_peak"],
                               "busy_frac": prof["mfma_busy_frac"],
                               "issued_over_algorithmic": prof["mfma_issued_flop_per_launch"] / prof_alg}
                              if prof and "mfma_busy_frac" in prof else None),
            "kernel": "moment_kernel", "algorithmic_tflops": r["moment_tflops"],
            "flop_per_launch": r["moment_flop_per_launch"], "inner_b": r["config"]["inner_b"],
            "ms_per_launch": r["moment_ms_per_launch"]}
    line = {
        "metric": METRIC,
        "value": r["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[main_p],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "b": b, "d_max": d_max, "t": t, "prec": main_p,
                   "alg_flop_per_step": flops, "unique_flop_per_step": uflops},
        "roofline": roof,
        "paths": {p: {k: v for k, v in res[p].items()} for p in precs},
        "rel_err": {str(d): errs[d] for d in errs},
        "rel_err_other": {str(d): errs_other[d] for d in errs_other},
    }
    if not args.no_batched:
        log("batched workload")
        line["batched"] = bench_batched(torch, pc, main_p, max(3, args.steps // 4), 1, not args.no_tune)
        log(f"  batched: {line['batched']['datasets_per_s']:.0f} datasets/s vs "
            f"{line['batched']['per_dataset_calls']['datasets_per_s']:.0f} with one call per dataset")
        line["batched"]["other_precisions"] = {
            "f16x2": bench_batched(torch, pc, "f16x2", max(3, args.steps // 4), 1, not args.no_tune, per_dataset=False)}
        log(f"  batched f16x2: {line['batched']['other_precisions']['f16x2']['datasets_per_s']:.0f} datasets/s")
    if not args.no_streaming:
        log("streaming window")
        sw = bench_streaming(torch, pc, X, n, d_max, b, main_p, max(5, args.steps // 2))
        line["streaming"] = sw
        log(f"  slide of 2 x {sw['batch']} samples: {sw['ms_per_slide']:.3f} ms ({sw['samples_per_s'] / 1e6:.1f} M samples/s, "
            f"{sw['update_tflops']:.1f} TFLOP/s); cumulants {sw['cumulants_ms']['recursion']:.3f} ms (recursion), "
            f"{sw['cumulants_ms']['moebius']:.3f} ms (general formula)")
        if main_p != "f16x2":
            sw16 = bench_streaming(torch, pc, X, n, d_max, b, "f16x2", max(5, args.steps // 2))
            line["streaming"]["other_precisions"] = {"f16x2": sw16}
            log(f"  slide in f16x2: {sw16['ms_per_slide']:.3f} ms")
    if not args.no_workloads:
        line["workloads"] = bench_workloads(torch, pc, max(5, args.steps // 2), not args.no_tune)
        line["small"] = bench_small(torch, pc, max(50, args.steps * 5), not args.no_tune)
        line["high_orders"] = bench_high_orders(torch, pc, max(5, args.steps // 2))
        log(f"  small workload: {line['small']['eager_us_per_call']:.1f} us per eager call, "
            f"{line['small']['graph_us_per_replay']:.1f} us per graph replay")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        import oracle as orc

        orc.build()
        line["cpu_baseline"] = cpu_baseline(orc, X, n, d_max, b, pc, args.cpu_seconds)
        line["cpu_baseline"]["other_workloads"] = cpu_oracle_configs(orc, pc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
