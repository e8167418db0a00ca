"""Parity of the shifted CholeskyQR3 schedule (Algorithm 5) with the oracle.

Bars, as for the other schedules:
* the accuracy bounds ||Q^T Q - I||_F <= 1e-13 and ||A - QR||_F / ||A||_F <=
  1e-14, R within 100 n u kappa of the oracle's R (relative Frobenius), Q
  within 100 n u kappa elementwise where kappa <= 1e6;
* scaled Hadamard input: Q = H and R = c I to a few units of roundoff (the
  shift is exact there, but Q1 = A R1^{-1} is rounded, so not bit for bit);
* the breakdown column exactly;
* fixed arguments give bitwise identical results.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402


def _factor(a, ld=None, check=True, b=0):
    q, r = cqr.qr(to_dev(a, ld), b=b, schedule="scqr3", check=check)
    torch.cuda.synchronize()
    return to_host(q), to_host(r)


def _check(a, q, r, kappa):
    n = a.shape[1]
    qo, ro = oracle.scqr3(a)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"scqr3 {a.shape}")
    if kappa <= 1e6:
        assert np.max(np.abs(q - qo)) <= 100 * n * U * kappa


@pytest.mark.parametrize("t,n,c", [(5, 32, 1.0), (6, 64, 4.0), (7, 128, 0.25), (6, 1, 2.0)])
def test_scaled_hadamard_closed_form(t, n, c):
    _, h, _ = matgen.hadamard_exact(4 ** t, n, seed=1)
    q, r = _factor(c * h)
    assert np.max(np.abs(q - h)) <= 16 * U * np.max(np.abs(h))
    assert np.max(np.abs(r - c * np.eye(n))) <= 16 * U * c
    assert np.all(np.tril(r, -1) == 0)


@pytest.mark.parametrize("kappa", [1.0, 1e5, 1e10, 1e12, 1e15])
@pytest.mark.parametrize("m,n", [(4096, 64), (5000, 100), (10000, 128), (2048, 16)])
def test_against_oracle(kappa, m, n):
    """Tile multiples and ragged tails (n = 100, m = 5000), up to the widest
    n the whole-matrix Cholesky holds; kappa up to 1e15 at these m, where the
    shifted Q1 stays within CholeskyQR2's reach."""
    a = matgen.test_matrix(m, n, kappa, seed=21)
    q, r = _factor(a)
    _check(a, q, r, kappa)


@pytest.mark.parametrize("m,n,ld", [(333, 1, None), (128, 128, None), (130, 128, 160),
                                    (1000, 77, 1003), (40000, 48, None)])
def test_edge_shapes(m, n, ld):
    """A single column, a square matrix, m just above n, padded strides, and a
    long m over many split-m chunks."""
    kappa = 1e8
    a = matgen.test_matrix(m, n, kappa, seed=22)
    q, r = _factor(a, ld)
    _check(a, q, r, kappa)


def test_cqr2_breaks_down_where_scqr3_does_not():
    """kappa = 1e12 at 4096 x 64: CholeskyQR2 (b = n under either panel
    schedule) breaks down on the GPU as in the oracle; sCQR3 meets the bounds."""
    a = matgen.test_matrix(4096, 64, 1e12, seed=1)
    with pytest.raises(cqr.Breakdown):
        q, r = cqr.qr(to_dev(a), b=64, schedule="mod")
    q, r = _factor(a)
    _check(a, q, r, 1e12)


def test_panel_argument_ignored_and_deterministic():
    a = matgen.test_matrix(6000, 96, 1e10, seed=23)
    q1, r1 = _factor(a)
    q2, r2 = _factor(a, b=16)
    q3, r3 = _factor(a, b=96)
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    assert np.array_equal(q1, q3) and np.array_equal(r1, r3)


def test_aliasing_stride_staged_bitwise():
    """lda = 8192 (a multiple of 1024 doubles) runs in the staging copy; the
    result equals the in-place run at lda + 16 bit for bit."""
    a = matgen.test_matrix(8192, 128, 1e12, seed=24)
    q1, r1 = _factor(a)
    q2, r2 = _factor(a, ld=8192 + 16)
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    _check(a, q1, r1, 1e12)


def test_in_place():
    a = matgen.test_matrix(4096, 64, 1e10, seed=25)
    ad = to_dev(a)
    q0, r0 = _factor(a)
    q, r = cqr.qr(ad, schedule="scqr3", out=(ad, cqr.empty_colmajor(64, 64, ad.device)))
    torch.cuda.synchronize()
    assert np.array_equal(to_host(q), q0) and np.array_equal(to_host(r), r0)


@pytest.mark.parametrize("col", [0, 13, 63])
def test_zero_column_breakdown(col):
    """A zero column passes the shifted Cholesky (its pivot is the shift) and
    leaves an exactly zero column in Q1; the first Cholesky of CholeskyQR2
    then fails at that column, on both sides."""
    a = matgen.test_matrix(4096, 64, 1e3, seed=26)
    a[:, col] = 0.0
    with pytest.raises(oracle.Breakdown) as eo:
        oracle.scqr3(a)
    with pytest.raises(cqr.Breakdown) as eg:
        _factor(a)
    assert eg.value.column == eo.value.column == col + 1


def test_nan_reaches_every_pivot():
    """A NaN entry makes ||A||_F^2, the shift and so every diagonal entry of
    W NaN: both sides fail at column 1."""
    a = matgen.test_matrix(4096, 32, 10.0, seed=27)
    a[1000, 9] = np.nan
    with pytest.raises(oracle.Breakdown) as eo:
        oracle.scqr3(a)
    with pytest.raises(cqr.Breakdown) as eg:
        _factor(a)
    assert eg.value.column == eo.value.column == 1


def test_full_size_properties():
    """The measured workload, 2^22 x 128 at kappa = 1e12, generated on the
    device: the bounds that hold at any size (orthogonality, residual, R
    upper triangular with a positive diagonal), and R against the GPU's
    mCQR2GS on the same matrix within 100 n u kappa."""
    from paper_2405_04237_amd import measure
    m, n, kappa = 1 << 22, 128, 1e12
    a = matgen.test_matrix_device(m, n, kappa, seed=31)
    q, r = cqr.qr(a, schedule="scqr3")
    torch.cuda.synchronize()
    assert measure.orthogonality(q) <= 1e-13
    assert measure.residual(a, q, r) <= 1e-14
    rh = to_host(r)
    assert np.all(np.tril(rh, -1) == 0) and np.all(np.diag(rh) > 0)
    del q
    q2, r2 = cqr.qr(a, b=32, schedule="mod")
    torch.cuda.synchronize()
    assert oracle.rel_fro(rh, to_host(r2)) <= 100 * n * U * kappa



def test_beyond_the_shift_reach():
    """2^18 x 32 at kappa = 1e16, past the reach of the shift of Algorithm 4
    at this m: the shifted Q1 keeps a condition number near 2.5e9, beyond
    CholeskyQR2's (section "Shifted CholeskyQR3"), and the oracle breaks
    down in its CholeskyQR2 stage. The GPU rounds in another order, so it may
    break down at another column or, by luck, get through; the contract is
    that it never returns info = 0 with factors outside the accuracy bounds:
    either info > 0, or ||Q^T Q - I||_F <= 1e-13 and the residual <= 1e-14."""
    m, n = 1 << 18, 32
    a = matgen.test_matrix(m, n, 1e16, seed=1)
    with pytest.raises(oracle.Breakdown):
        oracle.scqr3(a)
    ad = to_dev(a)
    ws = cqr.Workspace(m, n, 0, "scqr3", ad.device, lda=ad.stride(1))
    q, r = cqr.qr(ad, schedule="scqr3", workspace=ws, check=False)
    torch.cuda.synchronize()
    info = int(ws.info.item())
    if info > 0:
        print(f"GPU sCQR3 at kappa = 1e16: breakdown at column {info}")
        assert info <= n
        return
    qh, rh = to_host(q), to_host(r)
    orth, res = oracle.orthogonality(qh), oracle.residual(a, qh, rh)
    print(f"GPU sCQR3 at kappa = 1e16: info 0, orthogonality {orth:.2e}, residual {res:.2e}")
    assert info == 0
    assert orth <= 1e-13 and res <= 1e-14, (orth, res)
