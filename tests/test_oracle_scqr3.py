"""Pins of the oracle's shifted CholeskyQR (Algorithm 4) and shifted
CholeskyQR3 (Algorithm 5).

As for the other oracle pins, none of these compares the oracle with itself:
exact dyadic inputs give the shift, the shifted Cholesky factor and the final
factors in closed form; LAPACK's Householder QR fixes R; exact power-of-two
scaling and the exact zero column fix structural identities; the paper's
qualitative claims (sCQR3 stable where CholeskyQR2 breaks down) close the
set. A planted mistake in the shift must fail one of them.
"""
import importlib
import json
import math
import os

import numpy as np
import pytest

import matgen
import oracle

ocq = importlib.import_module("oracle.cholqr")

U = 2.0 ** -53
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))


def _scaled_hadamard(t, n, c):
    """c H with H the first n columns of the order-4^t Sylvester Hadamard
    matrix scaled to orthonormal columns (entries +-2^-t)."""
    _, h, _ = matgen.hadamard_exact(4 ** t, n, seed=1)
    return c * h, h


@pytest.mark.parametrize("t,n,c", [(5, 32, 1.0), (6, 32, 4.0), (7, 64, 0.25), (7, 1, 2.0)])
def test_shift_closed_form_on_scaled_hadamard(t, n, c):
    """For A = c H every step of Algorithm 4 is exact up to one square root:
    G = c^2 I, ||A||_F^2 = n c^2, sqrt(m) = 2^t, so s = 2^(t-53) n c^2 and
    W = (c^2 + s) I exactly; R1 = sqrt(c^2 + s) I with the correctly rounded
    square root. A wrong unit roundoff, a norm that is not squared, m in place
    of sqrt(m) or a shift added off the diagonal changes R1."""
    assert "sqrt(m) u ||A||_F^2" in GOLD["scqr_shift"]["formula"]
    a, h = _scaled_hadamard(t, n, c)
    s = 2.0 ** (t - 53) * n * c * c
    assert oracle.scqr_shift(a) == s
    q1, r1 = oracle.scqr(a)
    d = math.sqrt(c * c + s)
    assert d != c  # the shift is visible in the factor
    assert np.array_equal(r1, d * np.eye(n))
    assert np.array_equal(q1, a / d)


@pytest.mark.parametrize("t,n,c", [(5, 32, 1.0), (6, 48, 4.0), (7, 64, 0.25)])
def test_scqr3_recovers_scaled_hadamard(t, n, c):
    """CholeskyQR2 of Q1 = H c / sqrt(c^2 + s) undoes the shift: Q = H and
    R = c I to a few units of roundoff."""
    a, h = _scaled_hadamard(t, n, c)
    q, r = oracle.scqr3(a)
    assert np.max(np.abs(q - h)) <= 4 * U * np.max(np.abs(h))
    assert np.max(np.abs(r - c * np.eye(n))) <= 4 * U * c
    assert np.all(np.tril(r, -1) == 0)


@pytest.mark.parametrize("kappa", [1.0, 1e3, 1e8, 1e12, 1e15])
@pytest.mark.parametrize("m,n", [(2048, 48), (3000, 50), (9000, 100)])
def test_scqr3_against_householder(kappa, m, n):
    """R with a positive diagonal is unique: sCQR3's R agrees with LAPACK's
    Householder R within 100 n u kappa, and Q meets the orthogonality and
    residual bounds for every kappa up to 1e15."""
    a = matgen.test_matrix(m, n, kappa, seed=11)
    q, r = oracle.scqr3(a)
    _, rh = oracle.householder_qr(a)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert oracle.rel_fro(r, rh) <= 100 * n * U * kappa
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


@pytest.mark.parametrize("kappa", [1e12, 1e15])
def test_scqr3_stable_where_cqr2_breaks_down(kappa):
    """CholeskyQR2 breaks down beyond about u^-1/2; the shift lets sCQR
    factor up to O(u^-1) and leaves Q1 well enough conditioned (about
    u^-1/2) for the CholeskyQR2 that follows (subsection Shifted
    CholeskyQR3)."""
    assert GOLD["scqr_applicable_kappa"]["order"] == "u^-1"
    a = matgen.test_matrix(4096, 64, kappa, seed=1)
    with pytest.raises(oracle.Breakdown):
        oracle.cqr2(a)
    q1, _ = oracle.scqr(a)
    sv = np.linalg.svd(q1, compute_uv=False)
    assert sv[0] / sv[-1] <= 2.0 / math.sqrt(U)
    q, r = oracle.scqr3(a)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


def test_power_of_two_scaling_is_exact():
    """Scaling A by 2^k scales G and ||A||_F^2 by 4^k, so s by 4^k, R1 and R
    by 2^k, and leaves Q1 and Q unchanged, all bit for bit. A shift that is
    not quadratic in A breaks this."""
    a = matgen.test_matrix(5000, 40, 1e10, seed=4)
    q1, r1 = oracle.scqr(a)
    q, r = oracle.scqr3(a)
    for k in (-3, 5):
        f = 2.0 ** k
        assert oracle.scqr_shift(f * a) == f * f * oracle.scqr_shift(a)
        q1s, r1s = oracle.scqr(f * a)
        qs, rs = oracle.scqr3(f * a)
        assert np.array_equal(q1s, q1) and np.array_equal(r1s, f * r1)
        assert np.array_equal(qs, q) and np.array_equal(rs, f * r)


def test_zero_column_shift_succeeds_second_gram_breaks_down():
    """A zero column j keeps W positive definite (its pivot is the shift
    itself) but gives an exactly zero column of Q1, so the first Cholesky of
    CholeskyQR2 breaks down at column j + 1 (1-based)."""
    a = matgen.test_matrix(3000, 24, 1e3, seed=9)
    a[:, 13] = 0.0
    q1, r1 = oracle.scqr(a)
    assert r1[13, 13] == math.sqrt(oracle.scqr_shift(a))
    assert np.all(q1[:, 13] == 0.0)
    with pytest.raises(oracle.Breakdown) as ei:
        oracle.scqr3(a)
    assert ei.value.column == 14


def test_frobenius_sum_matches_exact_sum():
    """||X||_F^2 of small-integer entries is an exact integer sum; the chunked
    pairwise total must equal it (no row chunk dropped or counted twice)."""
    rng = np.random.default_rng(3)
    x = rng.integers(-8, 9, size=(3 * ocq.CHUNK + 77, 5)).astype(np.float64)
    assert oracle.frobenius_sq(x) == float(sum(int(v) * int(v) for v in x.ravel()))
    assert oracle.frobenius_sq(np.zeros((0, 3))) == 0.0


def test_cost_formula_scqr3_vs_cqr2():
    """The paper's sCQR3 count (5/3 n^3 + 6 m n^2 + 2 m n at P = 1) is about
    1.5 times CholeskyQR2's (n^3 + 4 m n^2) for m >> n."""
    from paper_2405_04237_amd.costs import scqr3_flops, cqr2_flops
    assert "6 m n^2" in GOLD["cost_scqr3"]["formula"]
    m, n = 4 * 1024 * 1024, 128
    assert scqr3_flops(m, n) == pytest.approx(5 * n ** 3 / 3 + 6 * m * n * n + 2 * m * n)
    assert scqr3_flops(m, n) / cqr2_flops(m, n) == pytest.approx(
        GOLD["scqr3_flops_over_cqr2"]["value"], rel=0.01)


def _mut_shift(kind):
    def f(x):
        m = x.shape[0]
        fro2 = ocq.frobenius_sq(x)
        if kind == "u_eps":
            return math.sqrt(m) * 2.0 ** -52 * fro2
        if kind == "m_not_sqrt":
            return m * ocq.UNIT_ROUNDOFF * fro2
        if kind == "norm_not_squared":
            return math.sqrt(m) * ocq.UNIT_ROUNDOFF * math.sqrt(fro2)
        return 0.0
    return f


@pytest.mark.parametrize("kind", ["u_eps", "m_not_sqrt", "norm_not_squared", "no_shift"])
def test_pins_catch_planted_shift_mistakes(monkeypatch, kind):
    """Each plausible mistake in the shift fails the Hadamard closed form or
    the kappa = 1e15 stability pin."""
    monkeypatch.setattr(ocq, "scqr_shift", _mut_shift(kind))
    caught = 0
    a, _ = _scaled_hadamard(6, 32, 4.0)
    s = 2.0 ** (6 - 53) * 32 * 16.0
    _, r1 = oracle.scqr(a)
    caught += not np.array_equal(r1, math.sqrt(16.0 + s) * np.eye(32))
    try:
        b = matgen.test_matrix(4096, 64, 1e15, seed=1)
        q, r = oracle.scqr3(b)
        caught += oracle.orthogonality(q) > 1e-13
    except oracle.Breakdown:
        caught += 1
    assert caught >= 1


def test_conservative_shift_reach_shrinks_with_m():
    """With W = A^T A + s I the shifted Q1 has singular values sigma_i /
    sqrt(sigma_i^2 + s), so kappa(Q1) is about sqrt(s) / sigma_min and grows
    like m^(1/4). At 2^18 rows and kappa = 1e16 that is about 2.5e9, past
    CholeskyQR2's reach: sCQR itself completes (the shift keeps W positive
    definite) and the CholeskyQR2 stage breaks down; the paper points to a
    smaller shift for such matrices."""
    a = matgen.test_matrix(1 << 18, 32, 1e16, seed=1)
    assert math.sqrt(oracle.scqr_shift(a)) * 1e16 > 1e9
    oracle.scqr(a)
    with pytest.raises(oracle.Breakdown):
        oracle.scqr3(a)
