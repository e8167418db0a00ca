"""Parity of the hand-written QR adjoint (cqr_backward) with the CPU oracle.

Bars: the GPU gradient and the oracle gradient, fed the same Q, R, dQ, dR,
agree within 100 n u kappa (relative Frobenius); the recompute mode (Q = A
R^{-1} applied implicitly) agrees with the stored-Q mode within the same
bound; central differences of L(A) = <dQ, Q(A)> + <dR, R(A)> at h = 1e-7
along a unit-Frobenius direction agree with <dA, E> within 1e-3 relative at
kappa = 1e6 (1e-6 at kappa = 1e2); n = 1 matches its closed form.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402
from paper_2405_04237_amd import autograd as cag  # noqa: E402


def _bwd(q, r, dq, dr, a=None, recompute=False):
    rd = to_dev(r)
    dqd = to_dev(dq) if dq is not None else None
    drd = to_dev(dr) if dr is not None else None
    if recompute:
        da = cag.qr_backward(rd, dq=dqd, dr=drd, a=to_dev(a))
    else:
        da = cag.qr_backward(rd, dq=dqd, dr=drd, q=to_dev(q))
    torch.cuda.synchronize()
    return to_host(da)


@pytest.mark.parametrize("m,n,kappa", [(4096, 64, 1e6), (5000, 37, 1e3), (2048, 128, 1e2)])
def test_adjoint_vs_oracle(m, n, kappa):
    a = matgen.test_matrix(m, n, kappa, seed=31)
    q, r = oracle.mcqr2gs(a, min(n, 32))
    dq, dr = matgen.cotangents(m, n, seed=31)
    ref = oracle.qr_adjoint(q, r, dq, dr)
    got = _bwd(q, r, dq, dr)
    assert oracle.rel_fro(got, ref) <= 100 * n * U * kappa
    rec = _bwd(q, r, dq, dr, a=a, recompute=True)
    assert oracle.rel_fro(rec, ref) <= 100 * n * U * kappa


def test_adjoint_missing_cotangents():
    m, n = 3000, 24
    a = matgen.test_matrix(m, n, 1e3, seed=2)
    q, r = oracle.householder_qr(a)
    dq, dr = matgen.cotangents(m, n, seed=2)
    for dqi, dri in ((dq, None), (None, dr)):
        ref = oracle.qr_adjoint(q, r, dqi, dri)
        got = _bwd(q, r, dqi, dri)
        assert oracle.rel_fro(got, ref) <= 100 * n * U * 1e3
    assert not _bwd(q, r, None, None).any()
    # the strict lower triangle of dR is ignored
    lower = dr + np.tril(np.ones((n, n)), -1)
    assert np.array_equal(_bwd(q, r, dq, lower), _bwd(q, r, dq, dr))


def test_adjoint_single_column_closed_form():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((3000, 1))
    dq = rng.standard_normal((3000, 1))
    dr = rng.standard_normal((1, 1))
    q, r = oracle.householder_qr(a)
    rr = r[0, 0]
    expect = (dq + q * (rr * dr[0, 0] - float(dq[:, 0] @ q[:, 0]))) / rr
    got = _bwd(q, r, dq, dr)
    assert np.max(np.abs(got - expect)) <= 1e-13 * np.max(np.abs(expect))


def _loss(ad, dq, dr):
    qd, rd = cqr.qr(ad, b=0, schedule="mod")
    q, r = to_host(qd), to_host(rd)
    return float(np.sum(dq * q) + np.sum(np.triu(dr) * r))


@pytest.mark.parametrize("m,n,kappa,tol", [(2048, 16, 1e2, 1e-6), (4096, 32, 1e6, 1e-3)])
def test_adjoint_central_differences(m, n, kappa, tol):
    a = matgen.test_matrix(m, n, kappa, seed=8)
    dq, dr = matgen.cotangents(m, n, seed=8)
    e = matgen.unit_direction(m, n, seed=8)
    qd, rd = cqr.qr(to_dev(a))
    da = cag.qr_backward(rd, dq=to_dev(dq), dr=to_dev(dr), q=qd)
    exact = float(np.sum(to_host(da) * e))
    h = 1e-7
    fd = (_loss(to_dev(a + h * e), dq, dr) - _loss(to_dev(a - h * e), dq, dr)) / (2 * h)
    assert abs(fd - exact) <= tol * abs(exact)


def test_autograd_function_matches_direct_call():
    m, n = 4096, 48
    a = matgen.test_matrix(m, n, 1e4, seed=5)
    dq, dr = matgen.cotangents(m, n, seed=5)
    for recompute in (False, True):
        ad = to_dev(a).requires_grad_(True)
        q, r = cag.qr_diff(ad, b=16, schedule="mod", recompute_q=recompute)
        loss = (q * to_dev(dq)).sum() + (r * to_dev(np.triu(dr))).sum()
        loss.backward()
        qd, rd = cqr.qr(to_dev(a), b=16, schedule="mod")
        if recompute:
            direct = cag.qr_backward(rd, dq=to_dev(dq), dr=to_dev(np.triu(dr)), a=to_dev(a))
        else:
            direct = cag.qr_backward(rd, dq=to_dev(dq), dr=to_dev(np.triu(dr)), q=qd)
        assert np.array_equal(to_host(ad.grad), to_host(direct))


def test_adjoint_batched_against_single_and_oracle():
    """64 x (32768 x 64), kappa = 1e4: the batched adjoint equals per-matrix
    calls (within rounding: the split-m plan differs) and the oracle."""
    bsz, m, n, kappa = 64, 32768, 64, 1e4
    qs, rs, dqs, drs, refs = [], [], [], [], []
    for i in range(bsz):
        a = matgen.test_matrix(m, n, kappa, seed=100 + i) if i < 4 else None
        if a is None:  # keep host time bounded: reuse four matrices, fresh cotangents
            a = matgen.test_matrix(m, n, kappa, seed=100 + i % 4)
        q, r = oracle.mcqr2gs(a, 32)
        dq, dr = matgen.cotangents(m, n, seed=100 + i)
        qs.append(q), rs.append(r), dqs.append(dq), drs.append(dr)
        if i % 16 == 0:
            refs.append((i, oracle.qr_adjoint(q, r, dq, dr)))

    def stack(ms):
        return torch.from_numpy(np.stack([np.ascontiguousarray(x.T) for x in ms])).to("cuda").transpose(1, 2)

    da = cag.qr_backward_batched(stack(rs), dq=stack(dqs), dr=stack(drs), q=stack(qs))
    torch.cuda.synchronize()
    for i, ref in refs:
        got = np.asfortranarray(da[i].cpu().numpy())
        assert oracle.rel_fro(got, ref) <= 100 * n * U * kappa
        single = _bwd(qs[i], rs[i], dqs[i], drs[i])
        assert oracle.rel_fro(got, single) <= 100 * n * U * kappa


def test_cfg5_full_size():
    """262144 x 128, kappa = 1e6, dQ, dR ~ N(0,1): GPU forward (mCQR2GS), GPU
    adjoint vs the oracle adjoint on the same Q, R; recompute mode; central
    differences with h = 1e-7."""
    m, n, kappa = 262144, 128, 1e6
    a = matgen.test_matrix(m, n, kappa, seed=55)
    dq, dr = matgen.cotangents(m, n, seed=55)
    ad = to_dev(a)
    qd, rd = cqr.qr(ad, b=0, schedule="mod")
    q, r = to_host(qd), to_host(rd)
    assert oracle.orthogonality(q) <= 1e-13
    ref = oracle.qr_adjoint(q, r, dq, dr)
    got = to_host(cag.qr_backward(rd, dq=to_dev(dq), dr=to_dev(dr), q=qd))
    assert oracle.rel_fro(got, ref) <= 100 * n * U * kappa
    rec = to_host(cag.qr_backward(rd, dq=to_dev(dq), dr=to_dev(dr), a=ad))
    assert oracle.rel_fro(rec, ref) <= 100 * n * U * kappa
    e = matgen.unit_direction(m, n, seed=55)
    h = 1e-7
    fd = (_loss(to_dev(a + h * e), dq, dr) - _loss(to_dev(a - h * e), dq, dr)) / (2 * h)
    exact = float(np.sum(got * e))
    assert abs(fd - exact) <= 1e-3 * abs(exact)


def test_adjoint_batched_n128_against_oracle():
    """4 x (8192 x 128), kappa = 1e3: the batched first pass of a 128-column
    adjoint (two balanced waves per row chunk, one matrix per grid row)
    against the oracle and per-matrix calls."""
    bsz, m, n, kappa = 4, 8192, 128, 1e3
    qs, rs, dqs, drs = [], [], [], []
    for i in range(bsz):
        a = matgen.test_matrix(m, n, kappa, seed=300 + i)
        q, r = oracle.mcqr2gs(a, 32)
        dq, dr = matgen.cotangents(m, n, seed=300 + i)
        qs.append(q), rs.append(r), dqs.append(dq), drs.append(dr)

    def stack(ms):
        return torch.from_numpy(np.stack([np.ascontiguousarray(x.T) for x in ms])).to("cuda").transpose(1, 2)

    da = cag.qr_backward_batched(stack(rs), dq=stack(dqs), dr=stack(drs), q=stack(qs))
    torch.cuda.synchronize()
    for i in range(bsz):
        got = np.asfortranarray(da[i].cpu().numpy())
        ref = oracle.qr_adjoint(qs[i], rs[i], dqs[i], drs[i])
        assert oracle.rel_fro(got, ref) <= 100 * n * U * kappa
        assert oracle.rel_fro(got, _bwd(qs[i], rs[i], dqs[i], drs[i])) <= 100 * n * U * kappa
