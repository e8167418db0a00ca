"""Panel-width autotuner with an accuracy gate.

The paper makes the panel width b the main tuning knob: narrower panels are
better conditioned (eq. cond_bounds) but cost more global reductions and
kernel launches (subsection "CholeskyQR2 with Gram-Schmidt", discussion of
Table 2). Here every candidate b is run on the caller's matrix; candidates
whose result misses the accuracy bounds (||Q^T Q - I||_F <= orth_tol,
||A - QR||_F / ||A||_F <= res_tol) or break down are discarded, and the
fastest remaining one wins. Results can be cached in a JSON file keyed on
(device, m bucket, n, schedule).
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


def candidates(n: int, schedule: str):
    c = [b for b in (16, 32, 64, 128, 256) if b <= min(n, _lib.CQR_MAX_PANEL)]
    return c or [n]


def _key(a, schedule):
    import torch
    m, n = a.shape
    name = torch.cuda.get_device_properties(a.device).name
    return f"{name}|m2^{int(round(math.log2(max(m, 1))))}|n{n}|{schedule}"


def tune(a, schedule: str = "mod", cands=None, reps: int = 2, cache: str | None = None,
         log=None):
    """Return (best_b, table) where table lists per-candidate time and accuracy."""
    import torch
    cache = cache or os.environ.get("CQR_TUNE_FILE")
    key = _key(a, schedule)
    if cache and os.path.exists(cache):
        d = json.load(open(cache))
        if key in d:
            return d[key]["b"], d[key]["table"]
    m, n = a.shape
    cands = cands or candidates(n, schedule)
    q = empty_colmajor(m, n, a.device, ld=a.stride(1))
    r = empty_colmajor(n, n, a.device)
    table = []
    for b in cands:
        ws = Workspace(m, n, b, schedule, a.device, lda=a.stride(1))
        row = {"b": b}
        try:
            qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws)
            row["orth"] = measure.orthogonality(q)
            row["res"] = measure.residual(a, q, r)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                qr(a, b=b, schedule=schedule, out=(q, r), workspace=ws, check=False)
            torch.cuda.synchronize()
            row["ms"] = (time.perf_counter() - t0) * 1e3 / reps
            row["ok"] = bool(row["orth"] <= ORTH_TOL and row["res"] <= RES_TOL
                             and int(ws.info.item()) == 0)
        except Breakdown as e:
            row.update(ok=False, breakdown=e.column)
        table.append(row)
        del ws
        if log:
            log(f"tune {schedule} b={b}: {row}")
    ok = [t for t in table if t.get("ok")]
    best = min(ok, key=lambda t: t["ms"])["b"] if ok else None
    if cache and best is not None:
        d = json.load(open(cache)) if os.path.exists(cache) else {}
        d[key] = {"b": best, "table": table}
        json.dump(d, open(cache, "w"), indent=1)
    return best, table
