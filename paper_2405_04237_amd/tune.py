"""Autotuner: panel width b behind an accuracy gate, then the kernel variants.

The paper makes the panel width b the main tuning knob: narrower panels are
better conditioned (eq. cond_bounds) but cost more global reductions and
kernel launches (subsection "CholeskyQR2 with Gram-Schmidt", discussion of
Table 2). On the GPU there are two more: the tile shape of the trailing
update (a 64-column slab of Y in LDS, 64 x 128 register tiles, or 32 x 64
tiles) and of the projections (64 x 128 or 64 x 64 tiles).

tune(): every candidate b is run on the caller's matrix; candidates whose
result misses the accuracy bounds (||Q^T Q - I||_F <= orth_tol,
||A - QR||_F / ||A||_F <= res_tol) or break down are discarded. For the
fastest remaining widths every tile variant is then timed; a variant must
reproduce the default variant's Q and R bit for bit (the kernels sum each
entry in the same order), so it cannot change the accuracy that passed the
gate. The fastest (b, update tile, projection tile) wins. Results can be
cached in a JSON file keyed on (device, m bucket, n, schedule).

tune_batched(): the batched form's panel width per column count: for each
column count of the batch in turn, every candidate b (at most 32, the
persistent kernel's limit) is tried with the other classes held at their
current choice; a candidate must leave every matrix of the batch unbroken and
within the accuracy bounds, and the fastest replay wins.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import Breakdown, Workspace, empty_colmajor, qr
from . import _lib, measure

ORTH_TOL = 1e-13
RES_TOL = 1e-14
UPDATE_TILES = ("resident", "slab", "wide", "narrow")
PROJ_TILES = ("wide", "narrow")


def candidates(n: int, schedule: str):
    c = [b for b in (16, 32, 64, 128, 256) if b <= min(n, _lib.CQR_MAX_PANEL)]
    return c or [n]


def _key(a, schedule):
    import torch
    m, n = a.shape
    name = torch.cuda.get_device_properties(a.device).name
    return f"{name}|m2^{int(round(math.log2(max(m, 1))))}|n{n}|{schedule}"


def _timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune(a, schedule: str = "mod", cands=None, reps: int = 2, cache: str | None = None,
         log=None, tiles: bool = True, finalists: int = 2):
    """Return (config, table): config = {"b", "update_tile", "proj_tile"} (None
    if no width passes the gate); table lists every run's time and accuracy."""
    import torch
    cache = cache or os.environ.get("CQR_TUNE_FILE")
    key = _key(a, schedule)
    if cache and os.path.exists(cache):
        d = json.load(open(cache))
        if key in d and "config" in d[key]:
            return d[key]["config"], d[key]["table"]
    m, n = a.shape
    cands = cands or candidates(n, schedule)
    q = empty_colmajor(m, n, a.device, ld=a.stride(1))
    r = empty_colmajor(n, n, a.device)
    table = []
    passed = []
    for b in cands:
        ws = Workspace(m, n, b, schedule, a.device, lda=a.stride(1))
        row = {"b": b, "update_tile": "auto", "proj_tile": "auto"}
        try:
            qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws)
            row["orth"] = measure.orthogonality(q)
            row["res"] = measure.residual(a, q, r)
            row["ms"] = _timed(lambda: qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws,
                                          check=False), reps)
            row["ok"] = bool(row["orth"] <= ORTH_TOL and row["res"] <= RES_TOL
                             and int(ws.info.item()) == 0)
        except Breakdown as e:
            row.update(ok=False, breakdown=e.column)
        table.append(row)
        if row["ok"]:
            passed.append(row)
        del ws
        if log:
            log(f"tune {schedule} b={b}: {row}")
    if not passed:
        return None, table
    best = min(passed, key=lambda t: t["ms"])
    if tiles:
        for base in sorted(passed, key=lambda t: t["ms"])[:finalists]:
            b = base["b"]
            ws = Workspace(m, n, b, schedule, a.device, lda=a.stride(1))
            qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws, check=False)
            q0, r0 = q.clone(), r.clone()
            for ut in UPDATE_TILES:
                if ut in ("slab", "resident") and b > 128:
                    continue  # these kernels hold at most 128 inner columns
                for pt in PROJ_TILES:
                    def run():
                        qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws, check=False,
                           update_tile=ut, proj_tile=pt)
                    run()
                    same = bool(torch.equal(q, q0) and torch.equal(r, r0))
                    row = {"b": b, "update_tile": ut, "proj_tile": pt, "orth": base["orth"],
                           "res": base["res"], "ms": _timed(run, reps),
                           "bitwise_equal_to_default": same, "ok": same}
                    table.append(row)
                    if same and row["ms"] < best["ms"]:
                        best = row
                    if log:
                        log(f"tune {schedule} b={b} update={ut} proj={pt}: {row['ms']:.3f} ms"
                            f"{'' if same else ' (NOT bitwise equal: discarded)'}")
            del ws, q0, r0
    config = {"b": best["b"], "update_tile": best["update_tile"], "proj_tile": best["proj_tile"]}
    if cache:
        d = json.load(open(cache)) if os.path.exists(cache) else {}
        d[key] = {"config": config, "table": table}
        json.dump(d, open(cache, "w"), indent=1)
    return config, table


def tune_batched(mats, bs, reps: int = 3, cands=(8, 16, 32), log=None):
    """Per column count, the fastest batched panel width whose replay keeps
    every matrix within the accuracy bounds. mats: column-major FP64 device
    matrices; bs: the starting widths (one per matrix). Returns (bs, table)."""
    import torch
    from . import BatchedCall

    ns = [a.shape[1] for a in mats]
    bs = list(bs)
    table = []

    def evaluate(trial):
        call = BatchedCall(mats, bs=trial)
        call.launch()
        torch.cuda.synchronize()
        broken = int((call.info != 0).sum().item())
        worst_o = worst_r = 0.0
        if not broken:
            for a, qq, rr in zip(mats, call.q, call.r):
                worst_o = max(worst_o, measure.orthogonality(qq))
                worst_r = max(worst_r, measure.residual(a, qq, rr))
        ok = broken == 0 and worst_o <= ORTH_TOL and worst_r <= RES_TOL
        ms = _timed(call.launch, reps)
        return {"ok": bool(ok), "breakdowns": broken, "max_orth": worst_o, "max_res": worst_r,
                "ms": ms}

    cur = evaluate(bs)
    table.append({"class": None, "bs": "start", **cur})
    for n in sorted(set(ns)):
        choice = None
        for b in cands:
            if b > min(n, 32):
                continue
            trial = [b if nn == n else bb for nn, bb in zip(ns, bs)]
            res = evaluate(trial)
            table.append({"class": n, "b": b, **res})
            if log:
                log(f"tune batched n={n} b={b}: {res}")
            if res["ok"] and (choice is None or res["ms"] < choice[1]["ms"]):
                choice = (trial, res)
        if choice is not None:
            bs = choice[0]
    return bs, table
