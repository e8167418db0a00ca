"""The plain entry points on the device: cqr_factor (the library's own
workspace and info word, read back with cqr_get_info) and cqr_backward with a
NULL workspace, against the same calls with a caller workspace (bit for bit:
the same kernels on the same operands), through a breakdown, a later call
that needs a larger workspace (grown in stream order, no host wait) and a
smaller call after it. Also the workspace query's leading dimension: an
aliasing lda with a non-aliasing m asks for the staging copy, and the staged
factorisation equals the in-place one bit for bit."""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402
from paper_2405_04237_amd import _lib  # noqa: E402


def _plain(ad, b):
    """cqr_factor on the current stream; returns (Q, R, info)."""
    m, n = ad.shape
    q = cqr.empty_colmajor(m, n, ad.device, ld=ad.stride(1))
    r = cqr.empty_colmajor(n, n, ad.device)
    stream = torch.cuda.current_stream(ad.device).cuda_stream
    _lib.check(_lib.factor(m, n, b, ad.data_ptr(), ad.stride(1), q.data_ptr(), r.data_ptr(), stream),
               "cqr_factor")
    info = _lib.get_info(stream)
    return q, r, info


@pytest.mark.parametrize("m,n,b,ld", [(4096, 64, 16, None), (1 << 18, 256, 64, None),
                                      (8000, 96, 32, 8192), (4096, 64, 16, None)])
def test_plain_factor_matches_ex(m, n, b, ld):
    a = matgen.test_matrix(m, n, 1e12, seed=81)
    ad = to_dev(a, ld)
    q, r, info = _plain(ad, b)
    assert info == 0
    q2, r2 = cqr.qr(ad, b=b, schedule="mod")
    torch.cuda.synchronize()
    assert torch.equal(q, q2) and torch.equal(r, r2)
    qh, rh = to_host(q), to_host(r)
    assert oracle.orthogonality(qh) <= 1e-13 and oracle.residual(a, qh, rh) <= 1e-14


def test_plain_factor_breakdown_then_success():
    a = matgen.test_matrix(4096, 32, 10.0, seed=82)
    bad = a.copy()
    bad[:, 19] = 0.0
    _, _, info = _plain(to_dev(bad), 8)
    assert info == 20
    q, r, info = _plain(to_dev(a), 8)   # the internal info word is reset per call
    assert info == 0
    assert oracle.orthogonality(to_host(q)) <= 1e-13


def test_plain_factor_grows_workspace_in_stream_order():
    """A small call, a much larger one queued right behind it (the library
    workspace grows: the stream waits for the small call, frees and
    reallocates), then the small one again, all without host waits in
    between; every result equals its caller-workspace twin."""
    shapes = [(4096, 64, 16), (1 << 20, 256, 64), (4096, 64, 16)]
    mats = [matgen.test_matrix(m, n, 1e10, seed=83 + i) for i, (m, n, b) in enumerate(shapes)]
    devs = [to_dev(a) for a in mats]
    stream = torch.cuda.current_stream().cuda_stream
    outs = []
    for ad, (m, n, b) in zip(devs, shapes):
        q = cqr.empty_colmajor(m, n, ad.device, ld=ad.stride(1))
        r = cqr.empty_colmajor(n, n, ad.device)
        _lib.check(_lib.factor(m, n, b, ad.data_ptr(), m, q.data_ptr(), r.data_ptr(), stream),
                   "cqr_factor")
        outs.append((q, r))
    assert _lib.get_info(stream) == 0
    for ad, (m, n, b), (q, r) in zip(devs, shapes, outs):
        q2, r2 = cqr.qr(ad, b=b, schedule="mod")
        torch.cuda.synchronize()
        assert torch.equal(q, q2) and torch.equal(r, r2), (m, n, b)


def test_backward_library_workspace_matches_caller_workspace():
    from paper_2405_04237_amd import autograd as cag
    stream = torch.cuda.current_stream().cuda_stream
    for m, n in ((4096, 32), (65536, 128), (4096, 32)):
        a = to_dev(matgen.test_matrix(m, n, 1e4, seed=84))
        q, r = cqr.qr(a)
        dq, dr = (to_dev(x) for x in matgen.cotangents(m, n, seed=84))
        ref = cag.qr_backward(r, dq=dq, dr=dr, q=q)
        da = cqr.empty_colmajor(m, n, a.device)
        _lib.check(_lib.backward(m, n, q.data_ptr(), 0, m, r.data_ptr(), dq.data_ptr(),
                                 dr.data_ptr(), da.data_ptr(), stream, None, 0), "cqr_backward")
        torch.cuda.synchronize()
        assert torch.equal(da, ref), (m, n)


def test_workspace_query_follows_lda():
    """m = 8000 stored with lda = 8192 (a multiple of 1024 doubles): the
    query with the leading dimension includes the staging copy, the query
    for lda = m does not; the staged run equals the in-place run at
    lda = 8016 bit for bit. And m = 8192 stored with lda = 8208 needs no
    staging room."""
    m, n, b = 8000, 96, 32
    with_stage = _lib.workspace_bytes(m, n, b, _lib.SCHED_MOD, 8192)
    plain = _lib.workspace_bytes(m, n, b, _lib.SCHED_MOD, m)
    assert with_stage - plain >= 8 * m * n
    assert (_lib.workspace_bytes(8192, n, b, _lib.SCHED_MOD, 8208)
            < _lib.workspace_bytes(8192, n, b, _lib.SCHED_MOD))
    a = matgen.test_matrix(m, n, 1e10, seed=85)
    q1, r1 = cqr.qr(to_dev(a, 8192), b=b)
    q2, r2 = cqr.qr(to_dev(a, 8016), b=b)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(q1), to_host(q2)) and np.array_equal(to_host(r1), to_host(r2))
