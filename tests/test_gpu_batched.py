"""Parity of the persistent batched factorisation with the CPU oracle.

Bars as for the single-matrix path: exact-arithmetic inputs bit for bit;
random inputs meet ||Q^T Q - I||_F <= 1e-13 and ||A - QR||_F / ||A||_F <=
1e-14 and match the oracle's mCQR2GS R within 100 n u kappa; a breakdown
column is reported exactly, per matrix; graph replays reproduce the eager
result bit for bit.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402

SHAPES = [(4096, 64, 16, 1e12), (5000, 128, 32, 1e14), (2048, 16, 16, 1e6), (7777, 100, 32, 1e10),
          (3000, 1, 1, 1.0), (12345, 33, 32, 1e8), (2100, 32, 8, 1e13), (65536, 128, 32, 1e14),
          (4500, 77, 20, 1e9), (16384, 64, 32, 1e15)]


def _check(a, q, r, b, kappa):
    n = a.shape[1]
    qo, ro = oracle.mcqr2gs(a, b)
    assert np.all(np.tril(r, -1) == 0) and np.all(np.diag(r) > 0)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"batched {a.shape} b={b}")


def test_batched_mixed_shapes():
    mats = [matgen.test_matrix(m, n, k, seed=200 + i) for i, (m, n, b, k) in enumerate(SHAPES)]
    qs, rs, info = cqr.qr_batched([to_dev(a) for a in mats], bs=[s[2] for s in SHAPES])
    torch.cuda.synchronize()
    assert not info.any()
    for a, q, r, (m, n, b, k) in zip(mats, qs, rs, SHAPES):
        _check(a, to_host(q), to_host(r), b, k)


def test_batched_hadamard_bitwise():
    cases = [(1024, 64, 16, 0), (4096, 40, 32, 37), (256, 16, 8, 5), (16384, 128, 32, 3)]
    mats, exp = [], []
    for i, (m, n, b, pad) in enumerate(cases):
        a, h, t = matgen.hadamard_exact(m, n, seed=10 + i, pad_rows=pad)
        mats.append(a), exp.append((h, t))
    qs, rs, info = cqr.qr_batched([to_dev(a) for a in mats], bs=[c[2] for c in cases])
    torch.cuda.synchronize()
    for q, r, (h, t) in zip(qs, rs, exp):
        assert np.array_equal(to_host(r), t)
        assert np.array_equal(to_host(q), h)


def test_batched_breakdown_is_per_matrix():
    mats = [matgen.test_matrix(3000, 24, 10.0, seed=i) for i in range(5)]
    mats[2][:, 13] = 0.0
    qs, rs, info = cqr.qr_batched([to_dev(a) for a in mats], bs=[8] * 5, check=False)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 0, 14, 0, 0]
    for i in (0, 1, 3, 4):
        _check(mats[i], to_host(qs[i]), to_host(rs[i]), 8, 10.0)


def test_batched_graph_replays_match_eager():
    mats = [to_dev(matgen.test_matrix(m, n, k, seed=300 + i)) for i, (m, n, b, k) in enumerate(SHAPES[:6])]
    call = cqr.BatchedCall(mats, bs=[s[2] for s in SHAPES[:6]])
    call.launch()
    torch.cuda.synchronize()
    ref_q = [q.clone() for q in call.q]
    ref_r = [r.clone() for r in call.r]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call.launch()
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for q in call.q:
            q.fill_(float("nan"))
        for r in call.r:
            r.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for q, r, q0, r0 in zip(call.q, call.r, ref_q, ref_r):
            assert torch.equal(q, q0) and torch.equal(r, r0)
        assert not call.info.any()


def test_batched_workload_shape_sample():
    """The 512-matrix workload's shape distribution (m in [2048, 65536], n in
    {16, 32, 64, 128}, b = min(ceil(n/2), 32), log10 kappa in [2, 14]): every matrix
    meets the accuracy bounds (measured on the device), a sample matches the
    oracle."""
    probs = matgen.batch_problems()
    mats = [to_dev(matgen.test_matrix(p.m, p.n, p.kappa, p.seed)) for p in probs]
    torch.cuda.synchronize()
    qs, rs, info = cqr.qr_batched(mats, bs=[p.b for p in probs])
    torch.cuda.synchronize()
    assert not info.any()
    from paper_2405_04237_amd import measure
    for a, q, r in zip(mats, qs, rs):
        assert measure.orthogonality(q) <= 1e-13
        assert measure.residual(a, q, r) <= 1e-14
    for i in range(0, len(probs), 64):
        p = probs[i]
        _check(to_host(mats[i]), to_host(qs[i]), to_host(rs[i]), p.b, p.kappa)


def test_batched_teams_breakdown_and_determinism():
    """Matrices are split by rows over a team of workgroups (a batch of eight
    on a device of hundreds of workgroups splits every matrix over sixteen
    workgroups of at least 128 rows; a large batch splits the matrices above
    a fair share over up to four). Every member takes the same Cholesky
    decisions, so a breakdown column is still reported exactly; team sums go
    through a fixed member order, so two runs agree bit for bit; the results
    meet the oracle bounds."""
    specs = [(65536, 128, 32, 1e12), (60000, 64, 32, 10.0)] + [(4096, 32, 16, 1e6)] * 6
    mats = [matgen.test_matrix(m, n, k, seed=700 + i) for i, (m, n, b, k) in enumerate(specs)]
    mats[1][:, 37] = 0.0
    runs = []
    for _ in range(2):
        qs, rs, info = cqr.qr_batched([to_dev(a) for a in mats], bs=[s[2] for s in specs], check=False)
        torch.cuda.synchronize()
        runs.append(([to_host(q) for q in qs], [to_host(r) for r in rs], info.cpu().tolist()))
    (q1, r1, i1), (q2, r2, i2) = runs
    assert i1 == i2 == [0, 38, 0, 0, 0, 0, 0, 0]
    for i in (0, 2, 3, 4, 5, 6, 7):
        assert np.array_equal(q1[i], q2[i]) and np.array_equal(r1[i], r2[i])
        _check(mats[i], q1[i], r1[i], specs[i][2], specs[i][3])


def test_batched_short_and_square():
    """Matrices far below the workload's 2048 rows: square (m = n = 128 and
    64), m just above n, a ragged panel width, and one narrow matrix, all in
    one launch (one workgroup each below 256 rows; the 1000 x 7 matrix is
    split over a team of seven 128-row shares)."""
    specs = [(128, 128, 32, 1e6), (200, 100, 25, 1e8), (64, 64, 16, 1e3), (1000, 7, 3, 1e2),
             (130, 128, 32, 1e10)]
    mats = [matgen.test_matrix(m, n, k, seed=900 + i) for i, (m, n, b, k) in enumerate(specs)]
    qs, rs, info = cqr.qr_batched([to_dev(a) for a in mats], bs=[s[2] for s in specs])
    torch.cuda.synchronize()
    assert not info.any()
    for a, q, r, (m, n, b, k) in zip(mats, qs, rs, specs):
        _check(a, to_host(q), to_host(r), b, k)


def test_batched_single_small_matrix_team():
    """One small matrix in a launch of hundreds of resident workgroups is
    split over a team of up to sixteen 128-row-or-larger shares (the
    latency form of the batched kernel): it meets the oracle bounds, two
    runs agree bit for bit, and a zero column is reported at its index."""
    m, n, b, kappa = 4096, 64, 16, 1e12
    a = matgen.test_matrix(m, n, kappa, seed=950)
    runs = []
    for _ in range(2):
        qs, rs, info = cqr.qr_batched([to_dev(a)], bs=[b])
        torch.cuda.synchronize()
        assert not info.any()
        runs.append((to_host(qs[0]), to_host(rs[0])))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    _check(a, runs[0][0], runs[0][1], b, kappa)
    z = np.array(a, copy=True)
    z[:, 40] = 0.0
    _, _, info = cqr.qr_batched([to_dev(z)], bs=[b], check=False)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [41]
