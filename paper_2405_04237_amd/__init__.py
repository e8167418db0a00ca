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

__all__ = ["qr", "qr_batched", "BatchPlan", "BatchedCall", "Breakdown", "CqrError",
           "empty_colmajor", "as_colmajor", "Workspace", "SCHEDULES"]


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
    """Device scratch and info word for repeated factorisations of one size
    and leading dimension (lda = m when not given)."""

    def __init__(self, m: int, n: int, b: int, schedule: str, device, lda: int | None = None):
        torch = _torch()
        self.sched = SCHEDULES[schedule]
        self.bytes = _lib.workspace_bytes(m, n, b, self.sched, m if lda is None else lda)
        if self.bytes == 0:
            raise ValueError("invalid sizes")
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.info = torch.zeros(1, dtype=torch.int32, device=device)


def qr(a, b: int = 0, schedule: str = "mod", check: bool = True, out=None,
       workspace: Workspace | None = None, lookahead: bool = False, adaptive: bool = False,
       update_tile: str = "auto", proj_tile: str = "auto"):
    """Thin QR of a tall-and-skinny FP64 matrix: returns (Q, R).

    schedule "mod" = mCQR2GS (Algorithm 9), "orig" = CQR2GS (Algorithm 7),
    "scqr3" = shifted CholeskyQR3 (Algorithm 5; whole matrix, n <= 256, b
    ignored). b = 0 picks libcqr's default panel width. lookahead=True runs
    each mCQR2GS panel's chain on a side stream, overlapped with the trailing
    update (bitwise the same result). adaptive=True leaves out a panel's
    repeated CholeskyQR or re-orthogonalisation update when it is within
    libcqr's tolerance of doing nothing (mCQR2GS only). update_tile and
    proj_tile pick the kernel variant of the updates ("slab", "resident",
    "wide", "narrow") and projections ("wide", "narrow"); "auto" is libcqr's
    default, and every variant gives the same bits. With check=True the call waits
    for the device and raises Breakdown if a Cholesky pivot failed;
    otherwise the caller reads ``workspace.info``.
    """
    torch = _torch()
    _check_input(a)
    if schedule not in SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(SCHEDULES)}")
    if update_tile not in _lib.TILES or proj_tile not in _lib.TILES:
        raise ValueError(f"tile variants must be one of {sorted(_lib.TILES)}")
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
        workspace = Workspace(m, n, b, schedule, a.device, lda=lda)
    stream = torch.cuda.current_stream(a.device).cuda_stream
    st = _lib.factor_ex(m, n, b, a.data_ptr(), lda, q.data_ptr(), r.data_ptr(), stream,
                        SCHEDULES[schedule], workspace.info.data_ptr(),
                        workspace.buf.data_ptr(), workspace.bytes, lookahead, adaptive,
                        _lib.TILES[update_tile], _lib.TILES[proj_tile])
    _lib.check(st, "cqr_factor_ex")
    if check:
        col = int(workspace.info.item())
        if col:
            raise Breakdown(col)
    return q, r


class BatchPlan:
    """Shapes, longest-first queue order and launch size of a batched call
    (cqr_plan_batched). Immutable; reusable for any matrices of these shapes."""

    def __init__(self, ms, ns, bs=None, schedule: str = "mod"):
        self.ms, self.ns = [int(x) for x in ms], [int(x) for x in ns]
        self.handle = _lib.plan_batched(self.ms, self.ns, bs, SCHEDULES[schedule])

    def __len__(self):
        return len(self.ms)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h:
            _lib.plan_destroy(h)


class BatchedCall:
    """Device argument arrays for repeated cqr_factor_batched launches on the
    same tensors (e.g. inside a captured HIP graph): launch() enqueues the
    queue reset and the persistent kernel and nothing else."""

    def __init__(self, mats, bs=None, plan: BatchPlan | None = None, out=None):
        torch = _torch()
        for a in mats:
            _check_input(a)
            if not (a.stride(0) == 1 and a.stride(1) >= max(1, a.shape[0])):
                raise ValueError("batched inputs must be column-major")
        dev = mats[0].device
        self.a = list(mats)
        self.plan = plan or BatchPlan([a.shape[0] for a in mats], [a.shape[1] for a in mats], bs)
        if out is None:
            self.q = [empty_colmajor(a.shape[0], a.shape[1], dev, ld=a.stride(1)) for a in mats]
            self.r = [empty_colmajor(a.shape[1], a.shape[1], dev) for a in mats]
        else:
            self.q, self.r = out
        i64 = torch.int64
        self.d_a = torch.tensor([a.data_ptr() for a in self.a], dtype=i64, device=dev)
        self.d_q = torch.tensor([q.data_ptr() for q in self.q], dtype=i64, device=dev)
        self.d_r = torch.tensor([r.data_ptr() for r in self.r], dtype=i64, device=dev)
        self.d_lda = torch.tensor([a.stride(1) for a in self.a], dtype=i64, device=dev)
        self.info = torch.zeros(len(self.a), dtype=torch.int32, device=dev)

    def launch(self):
        torch = _torch()
        stream = torch.cuda.current_stream(self.d_a.device).cuda_stream
        st = _lib.factor_batched(self.plan.handle, self.d_a.data_ptr(), self.d_lda.data_ptr(),
                                 self.d_q.data_ptr(), self.d_r.data_ptr(), self.info.data_ptr(),
                                 stream)
        _lib.check(st, "cqr_factor_batched")


def qr_batched(mats, bs=None, check: bool = True):
    """Factor a list of column-major FP64 device matrices of uneven shape in
    one persistent launch (mCQR2GS each). Returns (Qs, Rs, info)."""
    call = BatchedCall(mats, bs)
    call.launch()
    if check:
        bad = (call.info != 0).nonzero().flatten().tolist()
        if bad:
            raise Breakdown(int(call.info[bad[0]].item()))
    return call.q, call.r, call.info
