"""The timed configuration at its full size: 2^22 x 1024, kappa = 1e15,
mCQR2GS with b = 128 and lda = m + 16, the matrix and launch configuration
bench.py times. At this size the oracle cannot run in a test, so the checks
are the properties that hold at any size, measured on the device with
torch's own products: ||Q^T Q - I||_F <= 1e-13, ||A - QR||_F / ||A||_F <=
1e-14, R upper triangular with a positive diagonal, no breakdown; and the
staged layout (lda = m) gives the same factors bit for bit."""
import pytest

import matgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402
from paper_2405_04237_amd import measure  # noqa: E402


def test_timed_configuration_accuracy():
    m, n, b, kappa = 1 << 22, 1024, 128, 1e15
    dev = torch.device("cuda:0")
    torch.cuda.empty_cache()  # earlier full-size tests leave 32 GiB blocks cached
    a = matgen.test_matrix_device(m, n, kappa, 3, device=dev, ld=m + 16)
    ws = cqr.Workspace(m, n, b, "mod", dev, lda=a.stride(1))
    q = cqr.empty_colmajor(m, n, dev, ld=a.stride(1))
    r = cqr.empty_colmajor(n, n, dev)
    cqr.qr(a, b=b, schedule="mod", out=(q, r), workspace=ws)
    torch.cuda.synchronize()
    assert int(ws.info.item()) == 0
    assert measure.orthogonality(q) <= 1e-13
    assert measure.residual(a, q, r) <= 1e-14
    assert torch.all(torch.tril(r, -1) == 0) and torch.all(torch.diagonal(r) > 0)
    # the same matrix stored with lda = m runs in the staging copy
    q0, r0 = q.clone(), r.clone()
    del q
    a2 = torch.empty((n, m), dtype=torch.float64, device=dev).t()
    a2.copy_(a)
    del a
    q2, r2 = cqr.qr(a2, b=b, schedule="mod")
    torch.cuda.synchronize()
    assert torch.equal(r2, r0) and torch.equal(q2, q0)
    del a2, q2, q0, ws
    torch.cuda.empty_cache()
