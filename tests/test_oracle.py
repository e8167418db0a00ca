"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks it against an
independent library routine (LAPACK Householder QR), exact arithmetic
(Hadamard inputs, rational Gram + 50-digit Cholesky), closed forms, exact
IEEE identities, or the paper's printed qualitative claims.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import matgen
import oracle
import importlib
ocq = importlib.import_module("oracle.cholqr")

U = 2.0 ** -53
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))

SCHEDULES = {
    "orig": lambda a, b: oracle.cqr2gs(a, b),
    "mod": lambda a, b: oracle.mcqr2gs(a, b),
}


def _check_structure(r):
    assert np.all(np.tril(r, -1) == 0.0)
    assert np.all(np.diag(r) > 0)


# ---------------------------------------------------------------- Householder
@pytest.mark.parametrize("kappa", [1.0, 1e3, 1e6, 1e10])
@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("m,n,b", [(2048, 48, 16), (3000, 50, 20), (4096, 64, 64)])
def test_against_householder(kappa, sched, m, n, b):
    """R is unique (positive diagonal): it must agree with LAPACK's Householder
    R within 100 n u kappa (relative Frobenius), and Q, R meet the accuracy
    bounds ||Q^T Q - I||_F <= 1e-13 and ||A - QR||_F/||A||_F <= 1e-14."""
    if b == n and kappa > 1e6:
        pytest.skip("single panel = CholeskyQR2, stable only to ~1e8")
    a = matgen.test_matrix(m, n, kappa, seed=11)
    q, r = SCHEDULES[sched](a, b)
    qh, rh = oracle.householder_qr(a)
    _check_structure(r)
    assert oracle.rel_fro(r, rh) <= 100 * n * U * kappa
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    if kappa <= 1e3:  # Q is well determined: compare elementwise
        assert np.max(np.abs(q - qh)) <= 100 * n * U * kappa


def test_cqr2_against_householder():
    a = matgen.test_matrix(1000, 30, 1e4, seed=3)
    q, r = oracle.cqr2(a)
    qh, rh = oracle.householder_qr(a)
    assert oracle.rel_fro(r, rh) <= 100 * 30 * U * 1e4
    assert oracle.orthogonality(q) <= 1e-13


# ------------------------------------------------------------ exact inputs
@pytest.mark.parametrize("m,n,pad", [(1024, 64, 0), (4096, 40, 37), (256, 16, 5)])
def test_hadamard_exact(m, n, pad):
    """A = H T with exact arithmetic throughout: every algorithm must return
    Q = H and R = T bit for bit, whatever its panel width."""
    a, h, t = matgen.hadamard_exact(m, n, seed=5, pad_rows=pad)
    q, r = oracle.cqr(a)
    assert np.array_equal(q, h) and np.array_equal(r, t)
    q, r = oracle.cqr2(a)
    assert np.array_equal(q, h) and np.array_equal(r, t)
    for b in sorted({n, 16, 7, 1, max(1, n // 3)}):
        for name, f in SCHEDULES.items():
            q, r = f(a, b)
            assert np.array_equal(q, h), (name, b)
            assert np.array_equal(r, t), (name, b)
        q, r = oracle.cqrgs(a, b)
        assert np.array_equal(q, h) and np.array_equal(r, t)


def test_orthonormal_input():
    """Orthonormal columns give R = I (exactly for Hadamard columns)."""
    _, h, _ = matgen.hadamard_exact(1024, 32, seed=1)
    for f in SCHEDULES.values():
        q, r = f(h, 8)
        assert np.array_equal(r, np.eye(32)) and np.array_equal(q, h)
    # a Householder Q: R = I to a few ulps per entry
    a = matgen.test_matrix(2000, 24, 1.0, seed=2)
    qh, _ = oracle.householder_qr(a)
    for f in SCHEDULES.values():
        q, r = f(qh, 8)
        assert np.max(np.abs(r - np.eye(24))) <= 24 * 10 * U


def test_single_panel_is_cqr2_bitwise():
    """b = n removes the Gram-Schmidt loop: CQR2GS and mCQR2GS both reduce to
    CholeskyQR2 (subsection CholeskyQR2 with Gram-Schmidt, special case b = n)."""
    a = matgen.test_matrix(3000, 40, 1e5, seed=9)
    q2, r2 = oracle.cqr2(a)
    for f in SCHEDULES.values():
        q, r = f(a, 40)
        assert np.array_equal(q, q2) and np.array_equal(r, r2)
        q, r = f(a, 1000)  # b > n clamps to n
        assert np.array_equal(q, q2) and np.array_equal(r, r2)


# ---------------------------------------------------------------- brute force
def _exact_r(a):
    """R of the thin QR from the Gram matrix in exact rationals and its
    Cholesky factor in 50-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 50
    m, n = a.shape
    fa = [[Fraction(float(a[i, j])) for j in range(n)] for i in range(m)]
    g = [[sum((fa[k][i] * fa[k][j] for k in range(m)), Fraction(0)) for j in range(n)]
         for i in range(n)]
    w = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            w[i, j] = mp.mpf(g[i][j].numerator) / g[i][j].denominator
    r = mp.matrix(n, n)
    for j in range(n):
        s = w[j, j] - sum(r[k, j] ** 2 for k in range(j))
        r[j, j] = mp.sqrt(s)
        for c in range(j + 1, n):
            r[j, c] = (w[j, c] - sum(r[k, j] * r[k, c] for k in range(j))) / r[j, j]
    return np.array([[float(r[i, j]) for j in range(n)] for i in range(n)])


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("kappa", [1.0, 1e4, 1e7])
def test_bruteforce_small(n, kappa):
    m = 60
    a = matgen.test_matrix(m, n, kappa, seed=21 + n)
    rex = _exact_r(a)
    for b in range(1, n + 1):
        for f in SCHEDULES.values():
            _, r = f(a, b)
            assert oracle.rel_fro(r, rex) <= 10 * n * U * kappa, b


def test_single_column_closed_form():
    """n = 1: R = ||a||_2 and Q = a / ||a||_2."""
    rng = np.random.default_rng(0)
    a = np.asfortranarray(rng.standard_normal((5000, 1)) * 3.0)
    nrm = math.sqrt(math.fsum(a[:, 0] ** 2))
    for f in SCHEDULES.values():
        q, r = f(a, 1)
        assert abs(r[0, 0] - nrm) <= 8 * U * nrm
        assert np.max(np.abs(q[:, 0] - a[:, 0] / nrm)) <= 8 * U * np.max(np.abs(a)) / nrm


# ---------------------------------------------------------------- metamorphic
def test_metamorphic_bitwise():
    """Exact IEEE identities: scaling by 2^s, column sign flips D, and
    appending whole chunks of zero rows leave the factorisation equivariant
    bit for bit: (2^s A) -> (Q, 2^s R); (A D) -> (Q D, D R D); [A; 0] -> ([Q; 0], R)."""
    m, n, b = 2 * ocq.CHUNK, 24, 8
    a = matgen.test_matrix(m, n, 1e9, seed=4)
    d = np.where(np.random.default_rng(1).random(n) < 0.5, -1.0, 1.0)
    for f in SCHEDULES.values():
        q, r = f(a, b)
        q2, r2 = f(np.asfortranarray(a * 2.0 ** 7), b)
        assert np.array_equal(q2, q) and np.array_equal(r2, r * 2.0 ** 7)
        q3, r3 = f(np.asfortranarray(a * d), b)
        assert np.array_equal(q3, q * d) and np.array_equal(r3, d[:, None] * r * d)
        az = np.asfortranarray(np.vstack([a, np.zeros((ocq.CHUNK, n))]))
        q4, r4 = f(az, b)
        assert np.array_equal(r4, r) and np.array_equal(q4[:m], q) and not q4[m:].any()


# --------------------------------------------------------- invariants vs kappa
@pytest.mark.parametrize("kappa", [1.0, 1e5, 1e10, 1e12, 1e15])
def test_mod_invariants_cfg1_shape(kappa):
    """mCQR2GS keeps O(u) orthogonality and residual up to kappa = 1e15
    (subsection Modified CholeskyQR2 with Gram-Schmidt)."""
    a = matgen.test_matrix(4096, 64, kappa, seed=1)
    q, r = oracle.mcqr2gs(a, 16)
    _check_structure(r)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


@pytest.mark.parametrize("kappa", [1.0, 1e5, 1e10, 1e12])
def test_orig_invariants_cfg1_shape(kappa):
    a = matgen.test_matrix(4096, 64, kappa, seed=1)
    q, r = oracle.cqr2gs(a, 16)
    _check_structure(r)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


def test_mod_three_panels_at_1e15():
    """Three panels suffice for mCQR2GS at kappa = 1e15 on the paper's
    log-spaced spectrum (subsection Modified CholeskyQR2 with Gram-Schmidt);
    scaled down from 30000 x 3000 to 6000 x 300."""
    claim = GOLD["mcqr2gs_panels"]
    a = matgen.test_matrix(6000, 300, claim["three_panels_at_kappa"], seed=8)
    q, r = oracle.mcqr2gs(a, 100)
    assert oracle.orthogonality(q, normalised=True) <= 100 * U
    assert oracle.residual(a, q, r) <= 1e-14


# ---------------------------------------------------------- negative controls
def test_cqr2_breaks_down_beyond_its_limit():
    """CholeskyQR2 is stable only to kappa ~ 1e8 (section CholeskyQR2):
    at 1e12 the second-pass Gram is not numerically positive definite."""
    assert GOLD["cqr2_stability_limit_kappa"]["value"] == 1e8
    a = matgen.test_matrix(4096, 64, 1e12, seed=1)
    with pytest.raises(oracle.Breakdown) as ei:
        oracle.cqr2(a)
    assert 1 <= ei.value.column <= 64
    q, _ = oracle.cqr2(matgen.test_matrix(4096, 64, 1e6, seed=1))
    assert oracle.orthogonality(q) <= 1e-13


def test_orig_needs_narrow_panels_at_1e15():
    """CQR2GS loses orthogonality at kappa = 1e15 unless b is small (subsection
    CholeskyQR2 with Gram-Schmidt); mCQR2GS with the same b does not."""
    a = matgen.test_matrix(4096, 64, 1e15, seed=1)
    qo, _ = oracle.cqr2gs(a, 32)
    qm, _ = oracle.mcqr2gs(a, 32)
    assert oracle.orthogonality(qo) > 1e-13
    assert oracle.orthogonality(qm) <= 1e-13


def test_cqr_orthogonality_grows_like_kappa_squared():
    """Single-pass CholeskyQR loses orthogonality like u kappa^2 (section
    CholeskyQR): fitted log-log slope between 1.5 and 2.5 on [1e2, 1e6]."""
    ks = [1e2, 1e3, 1e4, 1e5, 1e6]
    vals = []
    for k in ks:
        a = matgen.test_matrix(4096, 32, k, seed=6)
        q, _ = oracle.cqr(a)
        vals.append(oracle.orthogonality(q))
    slope = np.polyfit(np.log10(ks), np.log10(vals), 1)[0]
    assert 1.5 < slope < 2.5, slope


def test_breakdown_reports_column():
    """A repeated column makes the Gram singular: breakdown at that column."""
    a = matgen.test_matrix(512, 8, 10.0, seed=2)
    a[:, 5] = a[:, 2]
    with pytest.raises(oracle.Breakdown) as ei:
        oracle.cqr(a)
    assert ei.value.column == 6
    a = matgen.test_matrix(512, 8, 10.0, seed=2)
    a[100, 3] = np.nan
    with pytest.raises(oracle.Breakdown) as ei:
        oracle.cqr(a)
    assert ei.value.column == 4


def test_panel_condition_interlacing():
    """eq. cond_bounds: kappa(A) >= kappa(B) >= s_{1+n-r} / s_r for a panel B
    of r columns (singular value interlacing)."""
    n, r = 40, 10
    a = matgen.test_matrix(800, n, 1e9, seed=3)
    s = np.linalg.svd(a, compute_uv=False)
    g = np.linalg.svd(a[:, :r], compute_uv=False)
    assert s[0] / s[-1] >= g[0] / g[-1] * (1 - 1e-6)
    assert g[0] / g[-1] >= s[n - r] / s[r - 1] * (1 - 1e-6)


# ------------------------------------------------------------ planted mistakes
def _mut_drop_last_chunk(f):
    def g(x, y):
        if x.shape[0] > ocq.CHUNK:
            k = (x.shape[0] - 1) // ocq.CHUNK * ocq.CHUNK
            return f(x[:k], y[:k])
        return f(x, y)
    return g


def _mut_solve_no_transpose(f):
    import scipy.linalg as sla
    return lambda x, u: sla.solve_triangular(u, x.T, trans="N", lower=False).T


MUTANTS = {
    # a dropped term: the last row chunk is left out of every X^T Y
    "xprod_drops_chunk": ("xprod", _mut_drop_last_chunk),
    # a wrong factor
    "xprod_half": ("xprod", lambda f: (lambda x, y: 0.5 * f(x, y))),
    # a wrong index: the right operand's columns shifted by one
    "xprod_shifted_column": ("xprod", lambda f: (lambda x, y: f(x, np.roll(y, 1, axis=1)))),
    # a transposed operand: Q = X U^{-T} instead of X U^{-1}
    "solve_transposed": ("_right_solve_upper", _mut_solve_no_transpose),
    # the wrong triangle: Q = X U instead of X U^{-1}
    "solve_with_u": ("_right_solve_upper", lambda f: (lambda x, u: x @ u)),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistakes(monkeypatch, mutant):
    """A plausible mistake planted in the oracle must fail a pin: the
    exact-Hadamard identity, the Householder cross-check or the accuracy
    bounds, for both schedules."""
    name, wrap = MUTANTS[mutant]
    monkeypatch.setattr(ocq, name, wrap(getattr(ocq, name)))
    a, h, t = matgen.hadamard_exact(4096, 32, seed=5, pad_rows=3000)
    ar = matgen.test_matrix(2 * ocq.CHUNK + 100, 32, 1e4, seed=7)
    _, rh = oracle.householder_qr(ar)
    for f in SCHEDULES.values():
        caught = 0
        try:
            q, r = f(a, 8)
            caught += not (np.array_equal(q, h) and np.array_equal(r, t))
            q, r = f(ar, 8)
            caught += oracle.rel_fro(r, rh) > 100 * 32 * U * 1e4
            caught += oracle.orthogonality(q) > 1e-13
        except (oracle.Breakdown, ValueError, np.linalg.LinAlgError):
            caught += 1
        assert caught >= 1


# ------------------------------------------------------------------ adjoint
def _loss(a, dq, dr):
    q, r = oracle.householder_qr(a)
    return float(np.sum(dq * q) + np.sum(np.triu(dr) * r))


@pytest.mark.parametrize("kappa", [1e1, 1e2])
def test_adjoint_finite_differences(kappa):
    """<dA, E> equals the directional derivative of L(A) = <dQ, Q> + <dR, R>
    (central differences; the error shrinks ~4x when h halves)."""
    m, n = 50, 6
    a = matgen.test_matrix(m, n, kappa, seed=31)
    dq, dr = matgen.cotangents(m, n, seed=31)
    e = matgen.unit_direction(m, n, seed=31)
    q, r = oracle.householder_qr(a)
    da = oracle.qr_adjoint(q, r, dq, dr)
    exact = float(np.sum(da * e))
    errs = []
    for h in (1e-3, 5e-4):
        fd = (_loss(a + h * e, dq, dr) - _loss(a - h * e, dq, dr)) / (2 * h)
        errs.append(abs(fd - exact))
    assert errs[1] <= 1e-5 * max(1.0, abs(exact)) * kappa
    assert errs[1] < errs[0] / 2.5  # second-order convergence


def test_adjoint_single_column_closed_form():
    """n = 1: dA = (dq + q (r dr - dq^T q)) / r with q = a / r."""
    rng = np.random.default_rng(4)
    a = rng.standard_normal((300, 1))
    dq = rng.standard_normal((300, 1))
    dr = rng.standard_normal((1, 1))
    q, r = oracle.householder_qr(a)
    rr = r[0, 0]
    expect = (dq + q * (rr * dr[0, 0] - float(dq[:, 0] @ q[:, 0]))) / rr
    got = oracle.qr_adjoint(q, r, dq, dr)
    assert np.max(np.abs(got - expect)) <= 1e-14 * np.max(np.abs(expect))


def test_adjoint_lower_dr_ignored_and_none_is_zero():
    a = matgen.test_matrix(80, 5, 10.0, seed=2)
    q, r = oracle.householder_qr(a)
    dq, dr = matgen.cotangents(80, 5, seed=2)
    full = dr + np.tril(np.ones((5, 5)), -1)
    assert np.array_equal(oracle.qr_adjoint(q, r, dq, full), oracle.qr_adjoint(q, r, dq, dr))
    assert np.array_equal(oracle.qr_adjoint(q, r, None, dr), oracle.qr_adjoint(q, r, np.zeros_like(dq), dr))


# ------------------------------------------------------------------ metrics
def test_metrics_on_exact_factorisation():
    a, h, t = matgen.hadamard_exact(1024, 16, seed=2)
    assert oracle.orthogonality(h) == 0.0
    assert oracle.residual(a, h, t) == 0.0
    # a known defect: scaling one column by (1 + d) gives ||Q^T Q - I||_F = 2d + d^2
    d = 2.0 ** -20
    hq = h.copy()
    hq[:, 3] *= 1 + d
    assert oracle.orthogonality(hq) == pytest.approx(2 * d + d * d, rel=1e-12)


def test_cost_formulas_match_paper_tables():
    """The flop model used for reporting reproduces Table 2's CQR2GS total and
    the Householder (PDGEQRF) count at P = 1."""
    from paper_2405_04237_amd.costs import cqr2gs_table2, householder_flops
    assert "4 m n^2" in GOLD["cost_cqr2gs"]["formula"]
    m, n, b = 4 * 1024 * 1024, 1024, 128
    assert cqr2gs_table2(m, n, b) == pytest.approx(2 * b * b * n / 3 + n ** 3 / 3 + 4 * m * n * n)
    assert householder_flops(m, n) == pytest.approx(2 * m * n * n - 2 * n ** 3 / 3)


def test_batched_workload_needs_two_panels():
    """The batched workload names b = min(n, 32); for n <= 32 that is a single
    panel, i.e. plain CholeskyQR2, which breaks down past kappa ~ 1e8 (section
    "CholeskyQR2"). On the workload's own n <= 32 matrices with kappa >= 1e10
    (a sample of eight of the smaller ones) the oracle's CholeskyQR2 breaks
    down on every one, while mCQR2GS with b = ceil(n / 2), the library's
    batched default, meets the accuracy bounds on every one."""
    import matgen
    probs = [p for p in matgen.batch_problems() if p.n <= 32 and p.kappa >= 1e10 and p.m <= 24000]
    assert len(probs) >= 8
    for p in probs[:8]:
        a = matgen.test_matrix(p.m, p.n, p.kappa, p.seed)
        with pytest.raises(oracle.Breakdown):
            oracle.cqr2(a)
        assert p.b == min((p.n + 1) // 2, 32)
        q, r = oracle.mcqr2gs(a, p.b)
        assert oracle.orthogonality(q) <= 1e-13 and oracle.residual(a, q, r) <= 1e-14
