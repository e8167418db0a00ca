#!/usr/bin/env python3
"""Benchmark: Householder-equivalent FP64 GFLOP/s of CholeskyQR2 with block
Gram-Schmidt on one MI355X, with the accuracy at kappa = 1e15.

One step = one whole factorisation A = QR of the workload matrix (every
kernel of the schedule: Grams, split-m reductions, Cholesky + inverse,
Q = X U^{-1}, projections, updates, R bookkeeping). The input is generated
on the device before the timed region. value = (2 m n^2 - 2 n^3 / 3) /
(seconds per step) / 1e9, the Householder flop count the paper uses for
ScaLAPACK's PDGEQRF (section "Testing environment", subsection "Software").

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("FP64 GFLOP/s (2mn²−⅔n³) + ‖QᵀQ−I‖ at κ=1e15, "
          "m=2^22 n=1024; batched/bwd")
PEAK_FP64 = 78.6e12     # MI355X dense FP64 (matrix and vector), FLOP/s
PEAK_HBM = 8.0e12       # MI355X HBM3E, bytes/s

WORKLOADS = {
    # the configuration the metric is quoted on (one GPU's row block)
    "tsqr-2^22x1024-k1e15": dict(m=1 << 22, n=1024, kappa=1e15, b_cands=(64, 128, 256), seed=3),
    "tsqr-2^20x256-k1e15": dict(m=1 << 20, n=256, kappa=1e15, b_cands=(64,), seed=2),
    "tsqr-4096x64-k1e12": dict(m=4096, n=64, kappa=1e12, b_cands=(16,), seed=1),
}
DEFAULT_WORKLOAD = "tsqr-2^22x1024-k1e15"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    """Hash of the sources of the single-matrix path's kernels and their
    launch logic (the batched kernel's sources are not part of it)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "device_common.h", "cqr.hip"):
        h.update(open(os.path.join(ROOT, "paper_2405_04237_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kind: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_sha") != kernel_sha() or d.get("workload") != workload:
        return None
    k = d.get("per_launch", {}).get(kind)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def bench_batched(steps: int, warmup: int, tune_widths: bool = True):
    """The batched workload (512 matrices of uneven shape) in one persistent
    launch, captured in a HIP graph and replayed; inputs generated on the host
    (the recipe of matgen.batch_problems) and uploaded before timing.
    tune_widths = False keeps the default panel widths (profiler runs)."""
    import numpy as np
    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import measure
    probs = matgen.batch_problems()
    log(f"batched: generating {len(probs)} matrices on the host")
    mats = []
    for p in probs:
        a = matgen.test_matrix(p.m, p.n, p.kappa, p.seed)
        mats.append(torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").t())
    from paper_2405_04237_amd import tune
    if tune_widths:
        bs, tune_table = tune.tune_batched(mats, [p.b for p in probs], log=log)
    else:
        bs, tune_table = [p.b for p in probs], None
    chosen = {n: sorted({b for b, p in zip(bs, probs) if p.n == n}) for n in sorted({p.n for p in probs})}
    log(f"batched: panel widths per column count {chosen}")
    call = cqr.BatchedCall(mats, bs=bs)
    call.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            call.launch()
    torch.cuda.current_stream().wait_stream(st)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    hh = sum(2.0 * p.m * p.n ** 2 - 2.0 * p.n ** 3 / 3 for p in probs)
    nbytes = sum(24.0 * p.m * p.n + 24.0 * p.m * p.n ** 2 / b for p, b in zip(probs, bs))
    worst = max(measure.orthogonality(q) for q in call.q)
    info = int((call.info != 0).sum().item())
    return {"workload": f"{len(probs)} matrices, m in [2048, 65536], n in {{16,32,64,128}}, "
                        "b = min(ceil(n/2), 32), kappa log-uniform in [1e2, 1e14]",
            "ms": round(ms, 3), "value": round(hh / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
            "graph": True, "max_orthogonality": worst, "breakdowns": info,
            "panel_width_per_n": {str(k): v for k, v in chosen.items()}, "tune": tune_table,
            "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms * 1e-3) / 1e9, 1),
                         "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": round(nbytes / (ms * 1e-3) / PEAK_HBM, 4),
                         "bytes_model": "sum 24 m n + 24 m n^2 / b"}}


def bench_backward(steps: int, warmup: int):
    """The adjoint at 262144 x 128 (kappa 1e6) and batched 64 x 32768 x 64
    (kappa 1e4), dQ and dR ~ N(0, 1), Q and R from this library's forward."""
    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import autograd as cag
    from paper_2405_04237_amd.costs import backward_bytes, backward_flops

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {}
    m, n = 262144, 128
    a = torch.from_numpy(matgen.test_matrix(m, n, 1e6, seed=55).T.copy()).to("cuda").t()
    dq, dr = matgen.cotangents(m, n, seed=55)
    dq = torch.from_numpy(dq.T.copy()).to("cuda").t()
    dr = torch.from_numpy(dr.T.copy()).to("cuda").t()
    q, r = cqr.qr(a)
    for mode, kw in (("stored_q", {"q": q}), ("recompute_q", {"a": a})):
        ms = timed(lambda: cag.qr_backward(r, dq=dq, dr=dr, **kw))
        fl, by = backward_flops(m, n), backward_bytes(m, n)
        out[mode] = {"workload": f"{m} x {n}, kappa=1e6", "ms": round(ms, 4),
                     "tflops": round(fl / (ms * 1e-3) / 1e12, 3),
                     "gbs": round(by / (ms * 1e-3) / 1e9, 1),
                     "roofline": {"bound": "mfma", "frac": round(fl / (ms * 1e-3) / PEAK_FP64, 4)}}
    bsz, m2, n2 = 64, 32768, 64
    log("backward: generating the batched inputs")
    qs, rs = [], []
    for i in range(bsz):
        ai = matgen.test_matrix(m2, n2, 1e4, seed=500 + i) if i < 8 else None
        ai = ai if ai is not None else matgen.test_matrix(m2, n2, 1e4, seed=500 + i % 8)
        qi, ri = cqr.qr(torch.from_numpy(ai.T.copy()).to("cuda").t())
        qs.append(qi), rs.append(ri)
    Q = torch.stack(qs)
    R = torch.stack(rs)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    dQ = torch.randn((bsz, n2, m2), dtype=torch.float64, device="cuda", generator=g).transpose(1, 2)
    dR = torch.triu(torch.randn((bsz, n2, n2), dtype=torch.float64, device="cuda", generator=g))
    ms = timed(lambda: cag.qr_backward_batched(R, dq=dQ, dr=dR, q=Q))
    by = bsz * backward_bytes(m2, n2)
    out["batched"] = {"workload": f"{bsz} x ({m2} x {n2}), kappa=1e4", "ms": round(ms, 4),
                      "gbs": round(by / (ms * 1e-3) / 1e9, 1),
                      "roofline": {"bound": "hbm", "frac": round(by / (ms * 1e-3) / PEAK_HBM, 4)}}
    return out


def bench_scqr3(steps: int, warmup: int):
    """Shifted CholeskyQR3 (Algorithm 5) at 2^22 x 128, kappa = 1e12 (past
    CholeskyQR2's limit, within the shifted algorithm's reach at this m),
    beside mCQR2GS on the same matrix."""
    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import _lib, measure
    from paper_2405_04237_amd.costs import householder_flops, schedule_bytes, schedule_flops

    m, n, kappa = 1 << 22, 128, 1e12
    dev = torch.device("cuda:0")
    log(f"scqr3: generating A ({m} x {n}, kappa={kappa:.0e}) on the device")
    a = matgen.test_matrix_device(m, n, kappa, seed=31, device=dev, ld=m + 16)
    q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, dev)
    out = {"workload": f"{m} x {n}, kappa={kappa:.0e}, lda {m + 16}"}
    for sched, b in (("scqr3", 0), ("mod", 32)):
        ws = cqr.Workspace(m, n, b, sched, dev, lda=a.stride(1))

        def step():
            cqr.qr(a, b=b, schedule=sched, out=(q, r), workspace=ws, check=False)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        _lib.profile_reset()
        _lib.profile_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        _lib.profile_enable(False)
        ms = e0.elapsed_time(e1) / steps
        kern = {}
        for kind in _lib.KERNEL_KINDS:
            p = _lib.profile_query(kind)
            if p["launches"]:
                kern[kind] = {"ms_per_step": round(p["ms"] / steps, 3),
                              "tflops": round(p["flops"] / (p["ms"] * 1e-3) / 1e12, 2),
                              "gbs": round(p["bytes"] / (p["ms"] * 1e-3) / 1e9, 1)}
        res = {"ms": round(ms, 3), "b": int(_lib.default_panel(m, n, cqr.SCHEDULES[sched]) if not b else b),
               "gflops_hh": round(householder_flops(m, n) / (ms * 1e-3) / 1e9, 1),
               "tflops_algorithmic": round(schedule_flops(m, n, b or n, sched) / (ms * 1e-3) / 1e12, 2),
               "gbs_algorithmic": round(schedule_bytes(m, n, b or n, sched) / (ms * 1e-3) / 1e9, 1),
               "info": int(ws.info.item()),
               "orthogonality": measure.orthogonality(q), "residual": measure.residual(a, q, r),
               "kernels": kern}
        out[sched] = res
        log(f"scqr3 leg, {sched}: {ms:.3f} ms, orthogonality {res['orthogonality']:.2e}")
        del ws
    del a, q, r
    torch.cuda.empty_cache()
    return out


def bench_adaptive(steps: int, warmup: int):
    """The run-time choice of CholeskyQR repetitions (adaptive) against the
    plain mCQR2GS at 2^20 x 256, b = 64, lda = m + 16: at kappa = 1 every
    repetition is left out, at kappa = 1e5 none is."""
    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import measure

    m, n, b = 1 << 20, 256, 64
    dev = torch.device("cuda:0")
    out = {"workload": f"{m} x {n}, b = {b}, lda {m + 16}"}
    for kappa in (1.0, 1e5):
        a = matgen.test_matrix_device(m, n, kappa, seed=61, device=dev, ld=m + 16)
        q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
        r = cqr.empty_colmajor(n, n, dev)
        ws = cqr.Workspace(m, n, b, "mod", dev, lda=a.stride(1))
        res = {}
        for mode in (False, True):
            def step():
                cqr.qr(a, b=b, schedule="mod", out=(q, r), workspace=ws, check=False, adaptive=mode)

            for _ in range(warmup):
                step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                step()
            e1.record()
            torch.cuda.synchronize()
            res["adaptive" if mode else "plain"] = {
                "ms": round(e0.elapsed_time(e1) / steps, 3),
                "orthogonality": measure.orthogonality(q), "residual": measure.residual(a, q, r),
                "info": int(ws.info.item())}
        out[f"kappa={kappa:.0e}"] = res
        log(f"adaptive leg, kappa {kappa:.0e}: " + json.dumps({k: v["ms"] for k, v in res.items()}))
        del a, q, r, ws
    torch.cuda.empty_cache()
    return out


def bench_small_graph(steps: int):
    """The small single-matrix workload (4096 x 64, b = 16, kappa = 1e12):
    eager calls against replays of one HIP graph holding the whole
    factorisation (the launch-bound case)."""
    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd.costs import householder_flops

    m, n, b = 4096, 64, 16
    dev = torch.device("cuda:0")
    a = matgen.test_matrix_device(m, n, 1e12, seed=1, device=dev)
    ws = cqr.Workspace(m, n, b, "mod", dev)
    q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, dev)

    def step():
        cqr.qr(a, b=b, schedule="mod", out=(q, r), workspace=ws, check=False)

    reps = max(steps, 50)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / reps
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            step()
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph = e0.elapsed_time(e1) / reps
    # the same matrix through the persistent batched kernel: one launch (a
    # team of workgroups), panel reductions in local memory
    call = cqr.BatchedCall([a], bs=[b])
    for _ in range(3):
        call.launch()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        call.launch()
    e1.record()
    torch.cuda.synchronize()
    single = e0.elapsed_time(e1) / reps
    hf = householder_flops(m, n)
    log(f"small single matrix: eager {eager:.3f} ms, graph {graph:.3f} ms, "
        f"single launch {single:.3f} ms")
    return {"workload": f"{m} x {n}, b = {b}, kappa=1e12", "reps": reps,
            "eager_ms": round(eager, 4), "graph_ms": round(graph, 4),
            "single_launch_ms": round(single, 4),
            "eager_gflops_hh": round(hf / (eager * 1e-3) / 1e9, 1),
            "graph_gflops_hh": round(hf / (graph * 1e-3) / 1e9, 1),
            "single_launch_gflops_hh": round(hf / (single * 1e-3) / 1e9, 1),
            "info": int(ws.info.item()), "single_launch_info": int(call.info[0].item())}


def time_steps(torch, step, steps: int, stream):
    """Run `steps` steps back to back between two synchronisations, with a
    HIP event on `stream` between consecutive steps: mean (total time /
    steps, the paper's statistic) and median of the per-step times."""
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for i in range(steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    srt = sorted(per)
    med = srt[steps // 2] if steps % 2 else 0.5 * (srt[steps // 2 - 1] + srt[steps // 2])
    return {"mean_ms": evs[0].elapsed_time(evs[steps]) / steps, "median_ms": med,
            "min_ms": srt[0], "max_ms": srt[-1]}


def kernel_table(_lib, steps: int):
    """Per-class launches, time and rates from the library's HIP-event
    bracketing (cqr_profile_*), per step."""
    kern = {}
    for kind in _lib.KERNEL_KINDS:
        p = _lib.profile_query(kind)
        if p["launches"]:
            kern[kind] = {"launches_per_step": p["launches"] / steps,
                          "ms_per_step": p["ms"] / steps,
                          "avg_launch_us": 1e3 * p["ms"] / p["launches"],
                          "tflops": p["flops"] / (p["ms"] * 1e-3) / 1e12 if p["ms"] else 0.0,
                          "gbs": p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] else 0.0,
                          "flops_per_launch": p["flops"] / p["launches"],
                          "bytes_per_launch": p["bytes"] / p["launches"]}
    return kern


def bench_tsqr_legs(steps: int, warmup: int):
    """The two smaller single-matrix workloads under both panel schedules,
    each beside the oracle on the host:
    * 2^20 x 256, b = 64, kappa in {1e5, 1e10, 1e15} (HBM-bound: about 3.2e10
      bytes of compulsory traffic per factorisation);
    * 4096 x 64, b = 16, kappa = 1e12 (latency-bound: ~70 dependent launches),
      eager and as one HIP graph replay."""
    import numpy as np
    import torch
    import matgen
    import oracle
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import measure
    from paper_2405_04237_amd.costs import householder_flops, schedule_bytes, schedule_flops

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}
    m, n, b = 1 << 20, 256, 64
    for kappa in (1e5, 1e10, 1e15):
        a = matgen.test_matrix_device(m, n, kappa, seed=2, device=dev, ld=m + 16)
        q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
        r = cqr.empty_colmajor(n, n, dev)
        # the oracle on a row sample of the same recipe (2^18 rows)
        ah = matgen.test_matrix(1 << 18, n, kappa, seed=2)
        for sched in ("orig", "mod"):
            ws = cqr.Workspace(m, n, b, sched, dev, lda=a.stride(1))

            def step():
                cqr.qr(a, b=b, schedule=sched, out=(q, r), workspace=ws, check=False)

            for _ in range(warmup):
                step()
            tm = time_steps(torch, step, steps, stream)
            ms = tm["mean_ms"]
            by = schedule_bytes(m, n, b, sched)
            fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
            t0 = time.perf_counter()
            fo(ah, b)
            to = time.perf_counter() - t0
            res = {"ms": round(ms, 4), "median_ms": round(tm["median_ms"], 4),
                   "value": round(householder_flops(m, n) / (ms * 1e-3) / 1e9, 1),
                   "unit": "GFLOP/s", "info": int(ws.info.item()),
                   "orthogonality": measure.orthogonality(q), "residual": measure.residual(a, q, r),
                   "executed_tflops": round(schedule_flops(m, n, b, sched) / (ms * 1e-3) / 1e12, 2),
                   "roofline": {"bound": "hbm", "achieved": round(by / (ms * 1e-3) / 1e9, 1),
                                "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                "frac": round(by / (ms * 1e-3) / PEAK_HBM, 4),
                                "bytes_model": "compulsory bytes of every streaming step"},
                   "oracle": {"rows": 1 << 18, "s": round(to, 3),
                              "value": round(householder_flops(1 << 18, n) / to / 1e9, 2),
                              "unit": "GFLOP/s"}}
            out[f"2^20x256 {sched} kappa={kappa:.0e}"] = res
            log(f"2^20x256 {sched} kappa {kappa:.0e}: {ms:.3f} ms (median {tm['median_ms']:.3f}), "
                f"orthogonality {res['orthogonality']:.2e}, oracle {to:.2f} s on 2^18 rows")
            del ws
        del a, q, r, ah
    torch.cuda.empty_cache()
    m, n, b, kappa = 4096, 64, 16, 1e12
    a = matgen.test_matrix_device(m, n, kappa, seed=1, device=dev)
    ah = matgen.test_matrix(m, n, kappa, seed=1)
    q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, dev)
    reps = max(steps, 50)
    for sched in ("orig", "mod"):
        ws = cqr.Workspace(m, n, b, sched, dev, lda=a.stride(1))

        def step():
            cqr.qr(a, b=b, schedule=sched, out=(q, r), workspace=ws, check=False)

        for _ in range(3):
            step()
        eager = time_steps(torch, step, reps, stream)
        g = torch.cuda.CUDAGraph()
        s2 = torch.cuda.Stream()
        s2.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s2):
            with torch.cuda.graph(g, stream=s2):
                step()
        torch.cuda.current_stream().wait_stream(s2)
        for _ in range(3):
            g.replay()
        graph = time_steps(torch, g.replay, reps, stream)
        fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
        ts = []
        for _ in range(10):
            t0 = time.perf_counter()
            fo(ah, b)
            ts.append(time.perf_counter() - t0)
        hf = householder_flops(m, n)
        out[f"4096x64 {sched} kappa=1e12"] = {
            "eager_ms": round(eager["mean_ms"], 4), "eager_median_ms": round(eager["median_ms"], 4),
            "graph_ms": round(graph["mean_ms"], 4), "graph_median_ms": round(graph["median_ms"], 4),
            "value_graph": round(hf / (graph["mean_ms"] * 1e-3) / 1e9, 1), "unit": "GFLOP/s",
            "info": int(ws.info.item()), "orthogonality": measure.orthogonality(q),
            "oracle": {"mean_s": round(sum(ts) / len(ts), 5), "median_s": round(sorted(ts)[5], 5)}}
        log(f"4096x64 {sched}: eager {eager['mean_ms']:.3f} ms, graph {graph['mean_ms']:.3f} ms, "
            f"oracle {sum(ts) / len(ts) * 1e3:.2f} ms")
        del ws, g
    return out


def cpu_baseline(w: dict, b: int, schedule: str, rows: int):
    """The oracle, untuned, on a row sample of the workload (host cores)."""
    import numpy as np
    import matgen
    import oracle
    from paper_2405_04237_amd.costs import householder_flops
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 0) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    m, n = rows, w["n"]
    log(f"cpu baseline: generating {m}x{n}")
    a = matgen.test_matrix(m, n, w["kappa"], seed=w["seed"])
    f = oracle.mcqr2gs if schedule == "mod" else oracle.cqr2gs
    t0 = time.perf_counter()
    q, r = f(a, b)
    dt = time.perf_counter() - t0
    del q, r, a
    log(f"cpu baseline: {dt:.2f} s")
    return {"value": round(householder_flops(m, n) / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": int(cores), "kind": "oracle",
            "sample": f"oracle {'mCQR2GS' if schedule == 'mod' else 'CQR2GS'} on {m} x {n} "
                      f"(the first {m} of {w['m']} rows' shape), kappa={w['kappa']:.0e}, b={b}, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default="mod", choices=["mod", "orig"])
    ap.add_argument("--b", type=int, default=0, help="panel width (0 = autotune)")
    ap.add_argument("--update-tile", default="auto",
                    choices=["auto", "slab", "wide", "narrow", "resident"],
                    help="update kernel variant (auto: the autotuner's choice, or libcqr's "
                         "default when --b is given)")
    ap.add_argument("--proj-tile", default="auto", choices=["auto", "wide", "narrow"])
    ap.add_argument("--no-tile-tune", action="store_true",
                    help="tune the panel width only (default tile variants)")
    ap.add_argument("--cpu-rows", type=int, default=1 << 18)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and adjoint measurements")
    ap.add_argument("--input", default="kappa", choices=["kappa", "gaussian"],
                    help="kappa: the workload's U diag(sigma) V^T matrix; gaussian: N(0,1) "
                         "entries and no accuracy check (hardware-counter runs: same kernels "
                         "and launch shapes, no library QR in the profiled process)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="finish with one 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-staged", action="store_true",
                    help="skip the extra timing of the same matrix with lda = m")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched workload (its graph replay) and print its "
                         "JSON; with --no-tile-tune its panel widths are the defaults")
    ap.add_argument("--lda-pad", type=int, default=16,
                    help="store A and Q with leading dimension m + pad (0: lda = m, which "
                         "for m = 2^22 aliases cache sets and makes the library factor a "
                         "staging copy; that case is also timed when pad > 0)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(multi-GPU row sharding is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import matgen
    import paper_2405_04237_amd as cqr
    from paper_2405_04237_amd import _lib, measure, tune
    from paper_2405_04237_amd.costs import householder_flops, schedule_bytes, schedule_flops

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(3)
    _lib.lib()  # fail loudly if libcqr.so is missing
    dev = torch.device("cuda:0")
    if args.batched_only:
        out = {"batched": bench_batched(args.steps, args.warmup, tune_widths=not args.no_tile_tune)}
        if args.calibration_copy:
            x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
            y = torch.ones(1 << 27, dtype=torch.float64, device=dev)
            x.copy_(y)
            torch.cuda.synchronize()
            out["calibration_copy_bytes"] = 2 * 8 * (1 << 27)
        print(json.dumps(out), flush=True)
        return
    w = WORKLOADS[args.workload]
    m, n, kappa = w["m"], w["n"], w["kappa"]
    t0 = time.perf_counter()
    lda = m + args.lda_pad
    if args.input == "gaussian":
        log(f"workload {args.workload}: N(0,1) input ({m} x {n}, lda {lda}) on the device")
        a = matgen.gaussian_device(m, n, w["seed"], device=dev, ld=lda)
    else:
        log(f"workload {args.workload}: generating A ({m} x {n}, kappa={kappa:.0e}, lda {lda}) "
            "on the device")
        a = matgen.test_matrix_device(m, n, kappa, w["seed"], device=dev, ld=lda)
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f} s")

    ut, pt = args.update_tile, args.proj_tile
    if args.b:
        b, table = args.b, None
    else:
        cfg, table = tune.tune(a, args.schedule, cands=list(w["b_cands"]), log=log,
                               tiles=not args.no_tile_tune)
        if cfg is None:
            log("no candidate panel width met the accuracy gate; using the narrowest")
            b = min(w["b_cands"])
        else:
            b = cfg["b"]
            if ut == "auto":
                ut = cfg["update_tile"]
            if pt == "auto":
                pt = cfg["proj_tile"]
    ws = cqr.Workspace(m, n, b, args.schedule, dev, lda=a.stride(1))
    q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, dev)
    stream = torch.cuda.current_stream(dev)
    log(f"configuration: b={b} update_tile={ut} proj_tile={pt}")

    def step():
        cqr.qr(a, b=b, schedule=args.schedule, out=(q, r), workspace=ws, check=False,
               update_tile=ut, proj_tile=pt)

    # warmup with every kernel class bracketed by HIP events: the per-kernel
    # table, and which class dominates the step
    _lib.profile_select(None)
    _lib.profile_reset()
    _lib.profile_enable(True)
    args.warmup = max(1, args.warmup)
    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    kern = kernel_table(_lib, args.warmup)
    log("per-kernel (warmup): " + json.dumps({k: {kk: round(vv, 3) for kk, vv in v.items()}
                                               for k, v in kern.items()}))
    dom = max((k for k in kern if k in ("gram", "proj", "update", "update_long", "trsm")),
              key=lambda k: kern[k]["ms_per_step"])
    # the timed region: only the dominant class carries events (two records
    # per launch of it), so the step time is that of the plain library
    log(f"warmup done ({args.warmup} steps), timing {args.steps} steps at b={b}")
    _lib.profile_select([dom])
    _lib.profile_reset()
    _lib.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tm = time_steps(torch, step, args.steps, stream)
    wall = time.perf_counter() - t0
    _lib.profile_enable(False)
    _lib.profile_select(None)
    ms = tm["mean_ms"]
    info = int(ws.info.item())
    live = kernel_table(_lib, args.steps)
    kern[dom] = live[dom]
    kd = kern[dom]
    intensity = kd["flops_per_launch"] / kd["bytes_per_launch"]
    if intensity >= PEAK_FP64 / PEAK_HBM:
        roof = {"bound": "mfma", "achieved": round(kd["tflops"], 3), "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": round(kd["tflops"] * 1e12 / PEAK_FP64, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(kd["gbs"], 1), "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": round(kd["gbs"] * 1e9 / PEAK_HBM, 4)}
    roof["kernel"] = dom
    roof["avg_launch_us"] = round(kd["avg_launch_us"], 2)
    roof["traffic"] = traffic_for(dom, args.workload)

    if args.input == "gaussian":
        orth = res = None
        log(f"no accuracy check (gaussian input)  info {info}")
    else:
        orth = measure.orthogonality(q)
        res = measure.residual(a, q, r)
        log(f"orthogonality {orth:.3e}  residual {res:.3e}  info {info}")
    value = householder_flops(m, n) / (ms * 1e-3) / 1e9
    # the whole step against both peaks: the flops the schedule executes
    # (about twice the Householder count, so value tops out near half of
    # the FP64 peak) and its compulsory bytes (each operand of each
    # streaming step read once, each output written once)
    ex_fl = schedule_flops(m, n, b, args.schedule)
    ex_by = schedule_bytes(m, n, b, args.schedule)
    step_roof = {"executed_tflops": round(ex_fl / (ms * 1e-3) / 1e12, 2),
                 "frac_fp64_peak": round(ex_fl / (ms * 1e-3) / PEAK_FP64, 4),
                 "algorithmic_gbs": round(ex_by / (ms * 1e-3) / 1e9, 1),
                 "frac_hbm_peak": round(ex_by / (ms * 1e-3) / PEAK_HBM, 4),
                 "executed_over_householder": round(ex_fl / householder_flops(m, n), 3)}
    staged = None
    if args.lda_pad and not args.no_staged:
        # the same matrix stored with lda = m: the library factors a staging copy
        a2 = torch.empty((n, m), dtype=torch.float64, device=dev).t()
        a2.copy_(a)
        del q
        q = cqr.empty_colmajor(m, n, dev, ld=m)
        ws2 = cqr.Workspace(m, n, b, args.schedule, dev, lda=a2.stride(1))
        k2 = max(1, min(args.steps, 3))
        for i in range(1 + k2):
            if i == 1:
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            cqr.qr(a2, b=b, schedule=args.schedule, out=(q, r), workspace=ws2, check=False,
                   update_tile=ut, proj_tile=pt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms2 = e0.elapsed_time(e1) / k2
        staged = {"lda": m, "steps": k2, "ms_per_step": round(ms2, 3),
                  "value": round(householder_flops(m, n) / (ms2 * 1e-3) / 1e9, 2),
                  "info": int(ws2.info.item())}
        log(f"lda = m (staged copy): {ms2:.3f} ms/step")
        del a2, ws2

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "median_ms_per_step": round(tm["median_ms"], 3),
        "step_ms_range": [round(tm["min_ms"], 3), round(tm["max_ms"], 3)],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "lda": lda,
                   "kappa": kappa if args.input == "kappa" else None, "input": args.input, "b": b,
                   "schedule": "mCQR2GS" if args.schedule == "mod" else "CQR2GS",
                   "update_tile": ut, "proj_tile": pt},
        "orthogonality": orth, "orthogonality_normalised": None if orth is None else orth / math.sqrt(n), "residual": res,
        "info": info, "wall_s": round(wall, 3), "roofline": roof, "step_roofline": step_roof,
        "kernels": kern, "kernels_note": "per-class HIP-event times from the warmup steps, except the roofline kernel (timed region)",
        "tune": table, "lda_m": staged,
        "paper_context": {
            "note": "the paper's own figures, other hardware and shapes, with communication; "
                    "context only, not this metric's baseline",
            "speedup_over_scalapack_pdgeqrf": {"cpu_version": ">6x", "gpu_version": "80x",
                                               "workload": "weak scaling, 10000 x 3000 rows per rank"},
            "gpu_hardware": "NVIDIA A100 40 GB, 4 per node (1 to 12 nodes)",
            "mcqr2gs_gpu_1_node_ms": 71.78,
            "householder_equivalent_tflops_per_a100": 2.44},
    }
    del q, r, ws, a
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["batched"] = bench_batched(max(args.steps, 3), 1)
        log(f"batched: {out['batched']['ms']} ms")
        out["backward"] = bench_backward(max(args.steps, 5), 2)
        log("backward: " + json.dumps(out["backward"]))
        out["scqr3"] = bench_scqr3(max(args.steps, 5), 2)
        out["adaptive"] = bench_adaptive(max(args.steps, 5), 2)
        out["small_graph"] = bench_small_graph(args.steps)
        out["tsqr_legs"] = bench_tsqr_legs(max(args.steps, 10), 3)
    if args.calibration_copy:
        x = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        y = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        x.copy_(y)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = 2 * 8 * (1 << 27)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, b, args.schedule, min(args.cpu_rows, m))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
