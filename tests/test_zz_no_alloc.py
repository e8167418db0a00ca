"""cqr_factor_noalloc (the entry point that allocates nothing) against
cqr_factor_ex with a caller workspace, through the C ABI.

Two calls in a row share the library's fixed device array; the second is a
smaller input, so every region it reads must have been written by that call
and not left over from the first. Results must equal cqr_factor_ex's bit for
bit (same kernels, same split-m plan) and meet the accuracy bounds against the
oracle (Algorithms 7 and 9)."""
import numpy as np
import pytest

import matgen
import oracle
from paper_2405_04237_amd import _lib
from tests.util import U, check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

# (m, n, b, kappa, schedule): the larger call first, then a smaller, ragged one
CALLS = [(1 << 17, 128, 32, 1e12, _lib.SCHED_MOD),
         (5000, 48, 16, 1e8, _lib.SCHED_MOD),
         (20000, 64, 16, 1e10, _lib.SCHED_ORIG),
         (3001, 40, 8, 1e6, _lib.SCHED_ORIG)]


def _noalloc(a_dev, b, sched, ld):
    import torch
    m, n = a_dev.shape
    q = torch.empty((n, ld), dtype=torch.float64, device="cuda").t()[:m]
    r = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = _lib.factor_noalloc(m, n, b, a_dev.data_ptr(), ld, q.data_ptr(), r.data_ptr(), sched,
                             info.data_ptr(), stream)
    assert st == _lib.CQR_OK, _lib.status_string(st)
    return q, r, info


def _with_workspace(a_dev, b, sched, ld):
    import torch
    m, n = a_dev.shape
    q = torch.empty((n, ld), dtype=torch.float64, device="cuda").t()[:m]
    r = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    info = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    nbytes = _lib.workspace_bytes(m, n, b, sched, ld)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = _lib.factor_ex(m, n, b, a_dev.data_ptr(), ld, q.data_ptr(), r.data_ptr(), stream, sched,
                        info.data_ptr(), ws.data_ptr(), nbytes)
    assert st == _lib.CQR_OK, _lib.status_string(st)
    return q, r, info


@pytest.mark.parametrize("pair", [(0, 1), (2, 3)])
def test_noalloc_matches_workspace_entry_point(pair):
    import torch
    for i in pair:
        m, n, b, kappa, sched = CALLS[i]
        print(f"cqr_factor_noalloc {m}x{n} b={b} kappa={kappa:.0e} schedule={sched}", flush=True)
        a = matgen.test_matrix(m, n, kappa, seed=900 + i)
        ld = m + 3
        a_dev = to_dev(a, ld=ld)
        q1, r1, info1 = _noalloc(a_dev, b, sched, ld)
        q2, r2, info2 = _with_workspace(a_dev, b, sched, ld)
        torch.cuda.synchronize()
        assert int(info1.item()) == 0 and int(info2.item()) == 0
        q1h, r1h = to_host(q1), to_host(r1)
        assert np.array_equal(q1h, to_host(q2)) and np.array_equal(r1h, to_host(r2))
        f = oracle.mcqr2gs if sched == _lib.SCHED_MOD else oracle.cqr2gs
        qo, ro = f(a, b)
        orth, orth_o = oracle.orthogonality(q1h), oracle.orthogonality(qo)
        assert orth <= max(1e-13, 10 * orth_o), (orth, orth_o)
        assert oracle.residual(a, q1h, r1h) <= 1e-14
        check_r(r1h, ro, r_bars(a, ro, kappa), f"noalloc {m}x{n} b={b}")
        assert np.all(np.tril(r1h, -1) == 0) and np.all(np.diag(r1h) > 0)


def test_noalloc_reports_breakdown_and_rejects_oversize():
    import torch
    m, n, b = 4096, 32, 16
    a = matgen.test_matrix(m, n, 1e4, seed=950)
    a[:, 5] = 0.0  # a zero column: the first panel's Gram matrix is singular
    a_dev = to_dev(a)
    q, r, info = _noalloc(a_dev, b, _lib.SCHED_MOD, m)
    torch.cuda.synchronize()
    assert int(info.item()) == 6
    # a size whose workspace exceeds the fixed array: rejected before any launch
    big_m, big_n, big_b = 1 << 22, 1024, 128
    assert _lib.workspace_bytes(big_m, big_n, big_b, _lib.SCHED_MOD) > _lib.CQR_NOALLOC_SCRATCH_BYTES
    stream = torch.cuda.current_stream().cuda_stream
    info.fill_(-5)
    st = _lib.factor_noalloc(big_m, big_n, big_b, a_dev.data_ptr(), big_m, q.data_ptr(),
                             r.data_ptr(), _lib.SCHED_MOD, info.data_ptr(), stream)
    assert st == _lib.CQR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int(info.item()) == -5  # nothing was launched
    # then a good call still works
    a2 = matgen.test_matrix(m, n, 1e4, seed=951)
    a2_dev = to_dev(a2)
    q, r, info = _noalloc(a2_dev, b, _lib.SCHED_MOD, m)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert oracle.orthogonality(to_host(q)) <= 1e-13
    assert oracle.residual(a2, to_host(q), to_host(r)) <= 1e-14
