"""Flop and byte models of the factorisation (host arithmetic only).

* ``householder_flops``: the Householder QR count the paper uses for
  ScaLAPACK's PDGEQRF, 2mn^2 - 2n^3/3 at P = 1 (section "Testing
  environment", subsection "Software"). Throughput is reported as this count
  divided by time ("Householder-equivalent" FLOP/s).
* ``cqr2gs_table2``: Table 2's total for CQR2GS at P = 1.
* ``cqr2_flops`` and ``scqr3_flops``: Table 1's CholeskyQR2 count and the
  shifted CholeskyQR3 cost equation (subsection "Shifted CholeskyQR3"), both
  at P = 1.
* Per-step algorithmic counts, following Tables 1 and 2: a Gram of an m x w
  panel costs m w^2 (syrk), forming Q = X U^{-1} costs m w^2 (trsm), a
  projection Y = Q^T Z or an update Z -= Q Y with Q m x p and Z m x q costs
  2 m p q each. Bytes are the compulsory HBM traffic of each step: every
  operand read once and every output written once, 8 bytes per element.
"""
from __future__ import annotations


def householder_flops(m: int, n: int) -> float:
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def cqr2gs_table2(m: int, n: int, b: int) -> float:
    return 2.0 * b * b * n / 3.0 + n ** 3 / 3.0 + 4.0 * m * n * n


def cqr2_flops(m: int, n: int) -> float:
    return float(n) ** 3 + 4.0 * m * n * n


def scqr3_flops(m: int, n: int) -> float:
    return 5.0 * n ** 3 / 3.0 + 6.0 * m * n * n + 2.0 * m * n


def panels(n: int, b: int):
    b = max(1, min(b, n))
    return [(s, min(s + b, n)) for s in range(0, n, b)]


def step_flops(kind: str, m: int, p: int, q: int = 0) -> float:
    if kind in ("gram", "trsm"):
        return float(m) * p * p
    if kind in ("proj", "update"):
        return 2.0 * m * p * q
    raise ValueError(kind)


def step_bytes(kind: str, m: int, p: int, q: int = 0) -> float:
    if kind == "gram":
        return 8.0 * m * p
    if kind == "trsm":
        return 16.0 * m * p
    if kind == "proj":
        return 8.0 * m * (p + q)
    if kind == "update":
        return 8.0 * m * (p + 2 * q)
    raise ValueError(kind)


def schedule_steps(m: int, n: int, b: int, schedule: str):
    """The streaming steps (kind, m, p, q) one factorisation performs."""
    pan = panels(n, b)
    steps = []
    if schedule == "orig":
        for _ in range(2):
            for s, e in pan:
                w = e - s
                steps += [("gram", m, w, 0), ("trsm", m, w, 0)]
                if e < n:
                    steps += [("proj", m, w, n - e), ("update", m, w, n - e)]
    elif schedule == "mod":
        s, e = pan[0]
        w = e - s
        steps += [("gram", m, w, 0), ("trsm", m, w, 0)] * 2
        for j in range(1, len(pan)):
            ps, pe = pan[j - 1]
            s, e = pan[j]
            w = e - s
            steps += [("proj", m, pe - ps, n - s), ("update", m, pe - ps, n - s),
                      ("gram", m, w, 0), ("trsm", m, w, 0),
                      ("proj", m, s, w), ("update", m, s, w),
                      ("gram", m, w, 0), ("trsm", m, w, 0)]
    elif schedule == "scqr3":
        # sCQR, then CholeskyQR2 of its Q: three whole-matrix Gram + trsm passes
        steps += [("gram", m, n, 0), ("trsm", m, n, 0)] * 3
    else:
        raise ValueError(schedule)
    return steps


def schedule_flops(m: int, n: int, b: int, schedule: str) -> float:
    f = sum(step_flops(k, mm, p, q) for k, mm, p, q in schedule_steps(m, n, b, schedule))
    if schedule == "orig":
        f += n ** 3 / 3.0  # R = R2 R1
    elif schedule == "scqr3":
        f += 2.0 * n ** 3 / 3.0  # R = (R3 R2) R1
    return f


def schedule_bytes(m: int, n: int, b: int, schedule: str) -> float:
    return sum(step_bytes(k, mm, p, q) for k, mm, p, q in schedule_steps(m, n, b, schedule))


def backward_flops(m: int, n: int, recompute_q: bool = False) -> float:
    """Adjoint: dQ^T Q (2mn^2, lower half counted as mn^2), then
    (dQ + Q C) R^{-T} (2mn^2 + mn^2); recomputing Q = A R^{-1} adds mn^2 per
    pass that needs Q."""
    f = 4.0 * m * n * n
    if recompute_q:
        f += 2.0 * m * n * n
    return f


def backward_bytes(m: int, n: int) -> float:
    """Pass 1 reads dQ and Q; pass 2 reads dQ and Q and writes dA."""
    return 8.0 * m * n * 5
