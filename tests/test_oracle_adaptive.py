"""Pins of the oracle's run-time choice of CholeskyQR repetitions in
mCQR2GS (``mcqr2gs(adaptive=tol)``; the paper's conclusion proposes it as
future work).

Fixed by exact arithmetic (Hadamard inputs: Z = 0 and Q^T Q = I exactly, so
every repetition is left out and the result is still exact), by LAPACK's
Householder R, by the accuracy bounds, and by the rule itself: a left-out
step can only leave what the tolerance admits.
"""
import numpy as np
import pytest

import matgen
import oracle

U = 2.0 ** -53
TOL = 1e-14


@pytest.mark.parametrize("m,n,b,pad", [(1024, 64, 16, 0), (4096, 40, 8, 37)])
def test_hadamard_exact_with_every_repetition_left_out(m, n, b, pad):
    a, h, t = matgen.hadamard_exact(m, n, seed=5, pad_rows=pad)
    q, r = oracle.mcqr2gs(a, b, adaptive=TOL)
    assert np.array_equal(q, h) and np.array_equal(r, t)


@pytest.mark.parametrize("kappa", [1.0, 1e2, 1e3, 1e5, 1e15])
@pytest.mark.parametrize("m,n,b", [(4096, 64, 16), (6000, 100, 32)])
def test_adaptive_against_householder(kappa, m, n, b):
    a = matgen.test_matrix(m, n, kappa, seed=3)
    q, r = oracle.mcqr2gs(a, b, adaptive=TOL)
    _, rh = oracle.householder_qr(a)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert oracle.rel_fro(r, rh) <= 100 * n * U * kappa
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


def test_well_conditioned_input_leaves_repetitions_out():
    """kappa = 1: every Z is far below the tolerance and every repeated Gram
    within it of I, so the adaptive result differs from the plain one, and
    its orthogonality is what the rule admits (at most about panels x tol)."""
    a = matgen.test_matrix(4096, 64, 1.0, seed=4)
    q0, r0 = oracle.mcqr2gs(a, 16)
    q1, r1 = oracle.mcqr2gs(a, 16, adaptive=TOL)
    assert not np.array_equal(q0, q1)
    assert oracle.orthogonality(q1) <= 4 * TOL


def test_ill_conditioned_input_keeps_every_repetition():
    """kappa >= 1e5: the decisions never fire; the result is the plain one."""
    for kappa in (1e5, 1e15):
        a = matgen.test_matrix(4096, 64, kappa, seed=4)
        q0, r0 = oracle.mcqr2gs(a, 16)
        q1, r1 = oracle.mcqr2gs(a, 16, adaptive=TOL)
        assert np.array_equal(q0, q1) and np.array_equal(r0, r1)


def test_orthonormal_input_single_cholesky():
    """Orthonormal columns: the first Cholesky gives R ~ I and the repeated
    one is left out; Q equals the input to a few units of roundoff."""
    q0 = matgen.test_matrix(4096, 48, 1.0, seed=6)
    q, r = oracle.mcqr2gs(q0, 48, adaptive=TOL)
    assert np.max(np.abs(r - np.eye(48))) <= 64 * U
    assert np.max(np.abs(q - q0)) <= 64 * U
