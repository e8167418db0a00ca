"""Run-time choice of CholeskyQR repetitions in mCQR2GS (adaptive=True)
against the oracle's ``mcqr2gs(adaptive=1e-14)``.

The decisions are floating-point comparisons of norms the two sides sum in
different orders, so parity is checked where every decision has a wide
margin: kappa = 1 (every repeated Gram within ~1e-15 of I and every Z near
1e-16, so every repetition is left out on both sides) and kappa >= 1e5
(no decision fires, so the adaptive run equals the plain one bit for bit).
Exact Hadamard inputs stay exact.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402

TOL = 1e-14


@pytest.mark.parametrize("m,n,b,pad", [(1024, 64, 16, 0), (4096, 40, 8, 37),
                                       (16384, 256, 128, 5), (4096, 128, 64, 0)])
def test_hadamard_exact(m, n, b, pad):
    a, h, t = matgen.hadamard_exact(m, n, seed=5, pad_rows=pad)
    q, r = cqr.qr(to_dev(a), b=b, schedule="mod", adaptive=True)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(r), t) and np.array_equal(to_host(q), h)


@pytest.mark.parametrize("m,n,b", [(4096, 64, 16), (6000, 100, 32), (65536, 256, 64),
                                   (20000, 256, 128)])
def test_well_conditioned_against_oracle(m, n, b):
    a = matgen.test_matrix(m, n, 1.0, seed=51)
    ad = to_dev(a)
    q, r = cqr.qr(ad, b=b, schedule="mod", adaptive=True)
    q0, r0 = cqr.qr(ad, b=b, schedule="mod")
    torch.cuda.synchronize()
    assert not torch.equal(q, q0)  # repetitions were left out
    q, r = to_host(q), to_host(r)
    qo, ro = oracle.mcqr2gs(a, b, adaptive=TOL)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    assert oracle.rel_fro(r, ro) <= 100 * n * U
    assert np.max(np.abs(q - qo)) <= 100 * n * U


@pytest.mark.parametrize("kappa", [1e5, 1e15])
@pytest.mark.parametrize("m,n,b", [(4096, 64, 16), (65536, 256, 64)])
def test_ill_conditioned_equals_plain(kappa, m, n, b):
    a = matgen.test_matrix(m, n, kappa, seed=52)
    ad = to_dev(a)
    q1, r1 = cqr.qr(ad, b=b, schedule="mod", adaptive=True)
    q0, r0 = cqr.qr(ad, b=b, schedule="mod")
    torch.cuda.synchronize()
    assert torch.equal(q1, q0) and torch.equal(r1, r0)


def test_staged_and_lookahead_agree():
    """The staged copy (lda a multiple of 1024 doubles) multiplies by the
    identity where the in-place run leaves the product out, and the
    look-ahead runs the same decisions on its side stream: all bit for bit."""
    m, n, b = 8192, 96, 32
    a = matgen.test_matrix(m, n, 1.0, seed=53)
    q1, r1 = cqr.qr(to_dev(a), b=b, schedule="mod", adaptive=True)             # staged
    q2, r2 = cqr.qr(to_dev(a, m + 16), b=b, schedule="mod", adaptive=True)     # in place
    q3, r3 = cqr.qr(to_dev(a, m + 16), b=b, schedule="mod", adaptive=True, lookahead=True)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2) and torch.equal(r1, r2)
    assert torch.equal(q2, q3) and torch.equal(r2, r3)


def test_breakdown_column_with_adaptive():
    a = matgen.test_matrix(4096, 64, 10.0, seed=54)
    a[:, 21] = 0.0
    with pytest.raises(cqr.Breakdown) as e:
        cqr.qr(to_dev(a), b=16, schedule="mod", adaptive=True)
    assert e.value.column == 22
