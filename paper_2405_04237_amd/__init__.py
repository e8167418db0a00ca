"""MI355X-native CholeskyQR2 with block Gram-Schmidt (arXiv 2405.04237).

Python front end of libcqr. PyTorch supplies device memory and the current
HIP stream; every step of the factorisation runs in libcqr's HIP kernels.
There is no CPU path: without libcqr.so or a GPU these functions raise.

    Q, R = qr(A, b=0, schedule="mod")

A is an m x n float64 tensor on a ROCm device with m >= n. Column-major
input (stride (1, lda)) is used in place; other layouts are copied once.
"""
from __future__ import annotations

from . import _lib
from ._lib import CqrError, SCHEDULES

__all__ = ["qr", "Breakdown", "CqrError", "empty_colmajor", "as_colmajor", "Workspace",
           "SCHEDULES"]


class Breakdown(ArithmeticError):
    """A panel's Gram matrix was not numerically positive definite."""

    def __init__(self, column: int):
        super().__init__(f"Gram matrix not positive definite at column {column}")
        self.column = column


def _torch():
    import torch
    return torch


def empty_colmajor(m: int, n: int, device, ld: int | None = None):
    """Uninitialised float64 m x n tensor with stride (1, ld)."""
    torch = _torch()
    ld = max(1, m) if ld is None else ld
    return torch.empty((n, ld), dtype=torch.float64, device=device).t()[:m]


def as_colmajor(a):
    if a.stride(0) == 1 and a.stride(1) >= max(1, a.shape[0]):
        return a
    return a.t().contiguous().t()


def _check_input(a):
    torch = _torch()
    if a.dim() != 2:
        raise ValueError("A must be 2-D")
    if a.dtype != torch.float64:
        raise TypeError("A must be float64")
    if a.device.type != "cuda":
        raise ValueError("A must live on a ROCm GPU (no CPU path)")
    m, n = a.shape
    if n < 1 or m < n:
        raise ValueError("need m >= n >= 1")


class Workspace:
    """Device scratch and info word for repeated factorisations of one size."""

    def __init__(self, m: int, n: int, b: int, schedule: str, device):
        torch = _torch()
        self.sched = SCHEDULES[schedule]
        self.bytes = _lib.workspace_bytes(m, n, b, self.sched)
        if self.bytes == 0:
            raise ValueError("invalid sizes")
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.info = torch.zeros(1, dtype=torch.int32, device=device)


def qr(a, b: int = 0, schedule: str = "mod", check: bool = True, out=None,
       workspace: Workspace | None = None):
    """Thin QR of a tall-and-skinny FP64 matrix: returns (Q, R).

    schedule "mod" = mCQR2GS (Algorithm 9), "orig" = CQR2GS (Algorithm 7).
    b = 0 picks libcqr's default panel width. With check=True the call waits
    for the device and raises Breakdown if a Cholesky pivot failed;
    otherwise the caller reads ``workspace.info``.
    """
    torch = _torch()
    _check_input(a)
    if schedule not in SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(SCHEDULES)}")
    a = as_colmajor(a)
    m, n = a.shape
    lda = a.stride(1)
    if out is None:
        q = empty_colmajor(m, n, a.device, ld=lda)
        r = empty_colmajor(n, n, a.device)
    else:
        q, r = out
        if q.shape != (m, n) or q.stride() != (1, lda) or r.shape != (n, n) or r.stride() != (1, n):
            raise ValueError("out tensors must be column-major with Q's stride equal to A's")
    if workspace is None:
        workspace = Workspace(m, n, b, schedule, a.device)
    stream = torch.cuda.current_stream(a.device).cuda_stream
    st = _lib.factor_ex(m, n, b, a.data_ptr(), lda, q.data_ptr(), r.data_ptr(), stream,
                        SCHEDULES[schedule], workspace.info.data_ptr(),
                        workspace.buf.data_ptr(), workspace.bytes)
    _lib.check(st, "cqr_factor_ex")
    if check:
        col = int(workspace.info.item())
        if col:
            raise Breakdown(col)
    return q, r
