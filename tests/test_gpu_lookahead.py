"""Look-ahead (mCQR2GS with each panel's chain on a side stream, overlapped
with the trailing update of the panels after it).

The look-ahead runs the same kernels on the same operands in an order that
respects every data dependency, so its Q, R and breakdown column must equal
those of the plain run bit for bit, at every shape, and meet the oracle's
bounds.
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import U, check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402


def _both(ad, b, check=True):
    out = []
    for la in (False, True):
        q, r = cqr.qr(ad, b=b, schedule="mod", lookahead=la, check=check)
        torch.cuda.synchronize()
        out.append((q.clone(), r.clone()))
    return out


@pytest.mark.parametrize("m,n,b,kappa,ld", [
    (4096, 64, 16, 1e12, None),      # the small single-matrix workload
    (5000, 100, 32, 1e15, None),     # ragged m, ragged last panel
    (4096, 70, 7, 1e8, 4099),        # odd panel width and odd stride
    (8192, 96, 32, 1e10, None),      # stride a multiple of 1024: staged copy
    (65536, 256, 64, 1e15, None),
])
def test_lookahead_bitwise_equal_and_accurate(m, n, b, kappa, ld):
    a = matgen.test_matrix(m, n, kappa, seed=41)
    (q0, r0), (q1, r1) = _both(to_dev(a, ld), b)
    assert torch.equal(q0, q1) and torch.equal(r0, r1)
    q, r = to_host(q1), to_host(r1)
    qo, ro = oracle.mcqr2gs(a, b)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"lookahead {m}x{n} b={b}")


def test_lookahead_breakdown_column():
    a = matgen.test_matrix(4096, 64, 10.0, seed=42)
    a[:, 37] = 0.0
    with pytest.raises(cqr.Breakdown) as e:
        cqr.qr(to_dev(a), b=16, schedule="mod", lookahead=True)
    assert e.value.column == 38


def test_lookahead_in_place_and_repeated():
    a = matgen.test_matrix(4096, 96, 1e12, seed=43)
    q0, r0 = cqr.qr(to_dev(a), b=32, schedule="mod")
    for _ in range(2):
        ad = to_dev(a)
        q, r = cqr.qr(ad, b=32, schedule="mod", lookahead=True,
                      out=(ad, cqr.empty_colmajor(96, 96, ad.device)))
        torch.cuda.synchronize()
        assert torch.equal(q, q0) and torch.equal(r, r0)


def test_lookahead_full_size_bitwise():
    """The timed configuration, 2^22 x 1024 with b = 128 (N(0,1) input: any
    input serves a bitwise comparison of two schedules of the same kernels)."""
    m, n, b = 1 << 22, 1024, 128
    a = matgen.gaussian_device(m, n, seed=44)
    ws = cqr.Workspace(m, n, b, "mod", a.device)
    q = cqr.empty_colmajor(m, n, a.device)
    r0 = cqr.empty_colmajor(n, n, a.device)
    cqr.qr(a, b=b, schedule="mod", out=(q, r0), workspace=ws)
    torch.cuda.synchronize()
    q0 = q.clone()
    r1 = cqr.empty_colmajor(n, n, a.device)
    cqr.qr(a, b=b, schedule="mod", out=(q, r1), workspace=ws, lookahead=True)
    torch.cuda.synchronize()
    assert torch.equal(r0, r1)
    assert torch.equal(q, q0)
