"""Differentiable QR on top of libcqr: the forward is the CholeskyQR2-BCGS
factorisation, the backward the hand-written adjoint kernels
(cqr_backward / cqr_backward_batched). Argument marshalling only."""
from __future__ import annotations

from . import _lib, as_colmajor, empty_colmajor, qr


def _torch():
    import torch
    return torch


def _colmajor_ld(t, ld):
    """t as an m x n tensor with stride (1, ld) (a copy if needed)."""
    if t.stride(0) == 1 and t.stride(1) == ld:
        return t
    out = empty_colmajor(t.shape[0], t.shape[1], t.device, ld=ld)
    out.copy_(t)
    return out


def qr_backward(r, dq=None, dr=None, q=None, a=None):
    """dA for the thin QR A = QR given cotangents dQ, dR (either may be None).

    Pass Q (stored from the forward) or, to recompute, A: then Q = A R^{-1} is
    applied implicitly and never formed.
    """
    torch = _torch()
    s = q if q is not None else a
    if s is None:
        raise ValueError("need Q or A")
    m, n = s.shape
    s = as_colmajor(s)
    lda = s.stride(1)
    r = _colmajor_ld(r, n)
    dq = _colmajor_ld(dq, lda) if dq is not None else None
    dr = _colmajor_ld(dr, n) if dr is not None else None
    da = empty_colmajor(m, n, s.device, ld=lda)
    nbytes = _lib.backward_workspace_bytes(m, n, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=s.device)
    stream = torch.cuda.current_stream(s.device).cuda_stream
    st = _lib.backward(m, n, s.data_ptr() if q is not None else None,
                       s.data_ptr() if q is None else None, lda, r.data_ptr(),
                       dq.data_ptr() if dq is not None else None,
                       dr.data_ptr() if dr is not None else None, da.data_ptr(), stream,
                       ws.data_ptr(), nbytes)
    _lib.check(st, "cqr_backward")
    return da


def qr_backward_batched(r, dq=None, dr=None, q=None, a=None):
    """Batched adjoint. q/a/dq: (batch, m, n) tensors whose matrices are
    column-major (each batch[i] has stride (1, m)); r/dr: (batch, n, n)
    column-major per matrix. Returns dA of the same layout as q/a."""
    torch = _torch()
    s = q if q is not None else a
    bsz, m, n = s.shape

    def cm(t, rows):
        # (batch, rows, n) with per-matrix stride (1, rows): storage (batch, n, rows)
        if t.stride(1) == 1 and t.stride(2) == rows and t.stride(0) == rows * n:
            return t
        out = torch.empty((bsz, n, rows), dtype=torch.float64, device=t.device).transpose(1, 2)
        out.copy_(t)
        return out

    s = cm(s, m)
    r = cm(r, n)
    dq = cm(dq, m) if dq is not None else None
    dr = cm(dr, n) if dr is not None else None
    da = torch.empty((bsz, n, m), dtype=torch.float64, device=s.device).transpose(1, 2)
    nbytes = _lib.backward_workspace_bytes(m, n, bsz)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=s.device)
    stream = torch.cuda.current_stream(s.device).cuda_stream
    st = _lib.backward_batched(bsz, m, n, s.data_ptr() if q is not None else None,
                               s.data_ptr() if q is None else None, m, m * n, r.data_ptr(),
                               dq.data_ptr() if dq is not None else None,
                               dr.data_ptr() if dr is not None else None, da.data_ptr(), stream,
                               ws.data_ptr(), nbytes)
    _lib.check(st, "cqr_backward_batched")
    return da


def _function():
    torch = _torch()

    class CQRFunction(torch.autograd.Function):
        """(Q, R) = CholeskyQR2-BCGS(A) with the libcqr adjoint as backward.
        recompute_q=True saves A instead of Q (Q is recomputed implicitly)."""

        @staticmethod
        def forward(ctx, a, b=0, schedule="mod", recompute_q=False):
            q, r = qr(a, b=b, schedule=schedule)
            ctx.recompute = bool(recompute_q)
            ctx.save_for_backward(a if recompute_q else q, r)
            return q, r

        @staticmethod
        def backward(ctx, dq, dr):
            s, r = ctx.saved_tensors
            if ctx.recompute:
                da = qr_backward(r, dq=dq, dr=dr, a=s)
            else:
                da = qr_backward(r, dq=dq, dr=dr, q=s)
            return da, None, None, None

    return CQRFunction


_FN = None


def CQRFunction():
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN


def qr_diff(a, b: int = 0, schedule: str = "mod", recompute_q: bool = False):
    """Differentiable (Q, R) = qr(a)."""
    return CQRFunction().apply(a, b, schedule, recompute_q)
