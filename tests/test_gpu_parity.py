"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars (see the tolerance derivation in the design notes):
* exact-arithmetic (Hadamard) inputs: Q and R bit for bit;
* b = n: both schedules reduce to CholeskyQR2 -> GPU ORIG == GPU MOD bitwise;
* random inputs: the accuracy bounds ||Q^T Q - I||_F <= 1e-13 and
  ||A - QR||_F / ||A||_F <= 1e-14 (MOD always; ORIG wherever the oracle's
  ORIG meets them at the same shape, else within 10x of the oracle's
  orthogonality), R within 100 n u kappa of the oracle's R (relative
  Frobenius), Q within 100 n u kappa elementwise where kappa <= 1e6;
* integer outputs (the breakdown column) exactly.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402


def _factor(a, b, sched, ld=None, check=True):
    ad = to_dev(a, ld)
    q, r = cqr.qr(ad, b=b, schedule=sched, check=check)
    torch.cuda.synchronize()
    return to_host(q), to_host(r)


@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("m,n,pad,b", [(1024, 64, 0, 16), (1024, 64, 37, 7), (4096, 40, 5, 40),
                                       (256, 16, 0, 1), (4096, 128, 100, 128), (16384, 96, 3, 32)])
def test_hadamard_bitwise(sched, m, n, pad, b):
    a, h, t = matgen.hadamard_exact(m, n, seed=5, pad_rows=pad)
    q, r = _factor(a, b, sched)
    assert np.array_equal(r, t)
    assert np.array_equal(q, h)


@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("kappa", [1.0, 1e5, 1e12, 1e15])
def test_cfg1_shape_against_oracle(sched, kappa):
    """4096 x 64, b = 16 (the small single-matrix workload)."""
    m, n, b = 4096, 64, 16
    a = matgen.test_matrix(m, n, kappa, seed=1)
    q, r = _factor(a, b, sched)
    fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
    qo, ro = fo(a, b)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    orth, orth_o = oracle.orthogonality(q), oracle.orthogonality(qo)
    if sched == "mod" or orth_o <= 1e-13:
        assert orth <= 1e-13, (orth, orth_o)
    else:
        assert orth <= 10 * orth_o, (orth, orth_o)
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"{sched} 4096x64 kappa={kappa:.0e}")
    if kappa <= 1e6:
        assert np.max(np.abs(q - qo)) <= 100 * n * U * kappa


@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("m,n,b,ld", [(1000, 40, 16, 1000), (1000, 40, 16, 1013), (777, 77, 13, 800),
                                      (70000, 130, 64, 70001), (5000, 1, 1, 5000),
                                      (20000, 300, 128, 20000), (128, 128, 64, 128),
                                      (130, 128, 128, 131)])
def test_ragged_shapes(sched, m, n, b, ld):
    """Row counts off the 16/64-row tiles, odd leading dimensions (scalar
    loads), ragged last panels (also after 128-column panels), n = 1, a
    square matrix, and m just above n (one 128-row block of Q = X U^{-1}
    plus a two-row tail)."""
    kappa = 1e8
    a = matgen.test_matrix(m, n, kappa, seed=3)
    q, r = _factor(a, b, sched, ld=ld)
    fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
    qo, ro = fo(a, b)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"{sched} {m}x{n} b={b} ld={ld}")


def test_single_panel_schedules_agree_bitwise():
    """b = n: CQR2GS and mCQR2GS are both CholeskyQR2 (subsection CholeskyQR2
    with Gram-Schmidt, special case b = n)."""
    a = matgen.test_matrix(8192, 48, 1e6, seed=4)
    q1, r1 = _factor(a, 48, "orig")
    q2, r2 = _factor(a, 48, "mod")
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    q3, r3 = _factor(a, 500, "mod")  # b > n clamps to n
    assert np.array_equal(q3, q2) and np.array_equal(r3, r2)


def test_deterministic_and_in_place():
    a = matgen.test_matrix(50000, 96, 1e10, seed=6)
    q1, r1 = _factor(a, 32, "mod")
    q2, r2 = _factor(a, 32, "mod")
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    ad = to_dev(a)
    q3, r3 = cqr.qr(ad, b=32, schedule="mod", out=(ad, cqr.empty_colmajor(96, 96, ad.device)))
    torch.cuda.synchronize()
    assert np.array_equal(to_host(q3), q1) and np.array_equal(to_host(r3), r1)


@pytest.mark.parametrize("sched", ["orig", "mod"])
def test_aliasing_stride_staged_bitwise(sched):
    """lda a multiple of 1024 doubles is factored in a staging copy with a
    shifted stride. The split-m plan depends on m only, so Q and R equal the
    in-place runs (lda + 16; a caller workspace without room for the copy)
    bit for bit, and meet the oracle bounds."""
    m, n, b, kappa = 8192, 96, 32, 1e10
    a = matgen.test_matrix(m, n, kappa, seed=8)
    q1, r1 = _factor(a, b, sched)                 # lda = 8192: staged
    q2, r2 = _factor(a, b, sched, ld=m + 16)      # in place
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2)
    ad = to_dev(a)
    small = cqr.Workspace(m + 16, n, b, sched, ad.device)   # no staging room for m
    assert small.bytes < cqr._lib.workspace_bytes(m, n, b, cqr.SCHEDULES[sched])
    q3, r3 = cqr.qr(ad, b=b, schedule=sched, workspace=small)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(q3), q1) and np.array_equal(to_host(r3), r1)
    fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
    qo, ro = fo(a, b)
    assert oracle.orthogonality(q1) <= 1e-13
    assert oracle.residual(a, q1, r1) <= 1e-14
    assert oracle.rel_fro(r1, ro) <= 100 * n * U * kappa


@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("col", [0, 11, 31])
def test_breakdown_column(sched, col):
    """An exactly zero column stays zero through every projection and update
    and gives an exactly zero Cholesky pivot: libcqr reports the same 1-based
    column as the oracle (exact integer)."""
    a = matgen.test_matrix(4096, 32, 10.0, seed=2)
    a[:, col] = 0.0
    with pytest.raises(oracle.Breakdown) as eo:
        (oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs)(a, 8)
    with pytest.raises(cqr.Breakdown) as eg:
        _factor(a, 8, sched)
    assert eg.value.column == eo.value.column == col + 1


@pytest.mark.parametrize("sched", ["orig", "mod"])
def test_breakdown_nan(sched):
    """A NaN entry makes its column's pivot NaN, which is not > 0."""
    a = matgen.test_matrix(4096, 32, 10.0, seed=2)
    a[1000, 9] = np.nan
    with pytest.raises(oracle.Breakdown) as eo:
        (oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs)(a, 8)
    with pytest.raises(cqr.Breakdown) as eg:
        _factor(a, 8, sched)
    assert eg.value.column == eo.value.column == 10


def test_cqr2_breakdown_at_1e12_like_oracle():
    """b = n at kappa = 1e12 is CholeskyQR2 past its limit: both sides break
    down (section CholeskyQR2); the columns need not coincide."""
    a = matgen.test_matrix(4096, 64, 1e12, seed=1)
    with pytest.raises(oracle.Breakdown):
        oracle.cqr2(a)
    with pytest.raises(cqr.Breakdown):
        _factor(a, 64, "mod")


def test_info_resets_between_calls():
    ws = cqr.Workspace(4096, 16, 8, "mod", "cuda")
    bad = matgen.test_matrix(4096, 16, 10.0, seed=1)
    bad[:, 3] = 0.0
    with pytest.raises(cqr.Breakdown):
        cqr.qr(to_dev(bad), b=8, workspace=ws)
    good = matgen.test_matrix(4096, 16, 10.0, seed=1)
    q, r = cqr.qr(to_dev(good), b=8, workspace=ws)
    assert int(ws.info.item()) == 0


@pytest.mark.parametrize("sched", ["orig", "mod"])
@pytest.mark.parametrize("kappa", [1e5, 1e10, 1e15])
def test_cfg2_shape_against_oracle(sched, kappa):
    """2^20 x 256, b = 64, kappa in {1e5, 1e10, 1e15}: the at-scale workload."""
    m, n, b = 1 << 20, 256, 64
    a = matgen.test_matrix(m, n, kappa, seed=2)
    q, r = _factor(a, b, sched)
    fo = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
    qo, ro = fo(a, b)
    orth, orth_o = oracle.orthogonality(q), oracle.orthogonality(qo)
    if sched == "mod" or orth_o <= 1e-13:
        assert orth <= 1e-13, (orth, orth_o)
    else:
        assert orth <= 10 * orth_o, (orth, orth_o)
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"{sched} 2^20x256 kappa={kappa:.0e}")
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
