"""ctypes binding of libcqr (include/cqr.h): same names, argument marshalling only.

The shared library is loaded from this package directory. There is no
fallback: if libcqr.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcqr.so")

CQR_OK = 0
CQR_ERR_ARG = -1
CQR_ERR_HIP = -2
CQR_ERR_NOMEM = -3
CQR_ERR_WORKSPACE = -4
CQR_ERR_UNSUPPORTED = -5
CQR_MAX_PANEL = 256
CQR_NOALLOC_SCRATCH_BYTES = 128 << 20

SCHED_MOD = 0
SCHED_ORIG = 1
SCHED_SCQR3 = 2
SCHEDULES = {"mod": SCHED_MOD, "orig": SCHED_ORIG, "scqr3": SCHED_SCQR3}

KERNEL_KINDS = ["gram", "proj", "update", "trsm", "reduce", "chol", "small", "batched", "copy",
                "update_long"]

# Every symbol include/cqr.h declares, with its ctypes signature.
_I64, _VP, _DP = C.c_int64, C.c_void_p, C.c_void_p


class CqrOptions(C.Structure):
    _fields_ = [("schedule", C.c_int), ("d_info", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("lookahead", C.c_int), ("adaptive", C.c_int),
                ("update_tile", C.c_int), ("proj_tile", C.c_int)]


SIGNATURES = {
    "cqr_factor": (C.c_int, [_I64, _I64, _I64, _DP, _I64, _DP, _DP, _VP]),
    "cqr_factor_ex": (C.c_int, [_I64, _I64, _I64, _DP, _I64, _DP, _DP, _VP, C.POINTER(CqrOptions)]),
    "cqr_factor_noalloc": (C.c_int, [_I64, _I64, _I64, _DP, _I64, _DP, _DP, C.c_int, _VP, _VP]),
    "cqr_workspace_bytes": (C.c_size_t, [_I64, _I64, _I64, C.c_int]),
    "cqr_workspace_bytes_ld": (C.c_size_t, [_I64, _I64, _I64, _I64, C.c_int]),
    "cqr_default_panel": (C.c_int64, [_I64, _I64, C.c_int]),
    "cqr_get_info": (C.c_int, [_VP, C.POINTER(C.c_int)]),
    "cqr_status_string": (C.c_char_p, [C.c_int]),
    "cqr_profile_enable": (C.c_int, [C.c_int]),
    "cqr_profile_reset": (C.c_int, []),
    "cqr_profile_select": (C.c_int, [C.c_uint]),
    "cqr_profile_query": (C.c_int, [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "cqr_plan_batched": (C.c_int, [_I64, _VP, _VP, _VP, C.c_int, C.POINTER(C.c_void_p)]),
    "cqr_factor_batched": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "cqr_plan_destroy": (None, [_VP]),
    "cqr_backward_workspace_bytes": (C.c_size_t, [_I64, _I64, _I64]),
    "cqr_backward": (C.c_int, [_I64, _I64, _DP, _DP, _I64, _DP, _DP, _DP, _DP, _VP, _VP, C.c_size_t]),
    "cqr_backward_batched": (C.c_int, [_I64, _I64, _I64, _DP, _DP, _I64, _I64, _DP, _DP, _DP, _DP,
                                       _VP, _VP, C.c_size_t]),
}

_lib = None


class CqrError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcqr.so not built ({LIB_PATH}); run __graft_entry__.build()")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def status_string(status: int) -> str:
    return lib().cqr_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != CQR_OK:
        raise CqrError(status, where)


def workspace_bytes(m: int, n: int, b: int, schedule: int, lda: int | None = None) -> int:
    if lda is None:
        return int(lib().cqr_workspace_bytes(m, n, b, schedule))
    return int(lib().cqr_workspace_bytes_ld(m, n, b, lda, schedule))


def default_panel(m: int, n: int, schedule: int) -> int:
    return int(lib().cqr_default_panel(m, n, schedule))


TILES = {"auto": 0, "slab": 1, "wide": 2, "narrow": 3, "resident": 4}


def factor_ex(m, n, b, a_ptr, lda, q_ptr, r_ptr, stream, schedule, info_ptr, ws_ptr, ws_bytes,
              lookahead=False, adaptive=False, update_tile=0, proj_tile=0):
    opt = CqrOptions(schedule, info_ptr, ws_ptr, ws_bytes, 1 if lookahead else 0,
                     1 if adaptive else 0, int(update_tile), int(proj_tile))
    return int(lib().cqr_factor_ex(m, n, b, a_ptr, lda, q_ptr, r_ptr, stream, C.byref(opt)))


def factor(m, n, b, a_ptr, lda, q_ptr, r_ptr, stream):
    return int(lib().cqr_factor(m, n, b, a_ptr, lda, q_ptr, r_ptr, stream))


def factor_noalloc(m, n, b, a_ptr, lda, q_ptr, r_ptr, schedule, info_ptr, stream):
    return int(lib().cqr_factor_noalloc(m, n, b, a_ptr, lda, q_ptr, r_ptr, schedule, info_ptr,
                                        stream))


def backward_workspace_bytes(m: int, n: int, batch: int = 1) -> int:
    return int(lib().cqr_backward_workspace_bytes(m, n, batch))


def backward(m, n, q_ptr, a_ptr, lda, r_ptr, dq_ptr, dr_ptr, da_ptr, stream, ws_ptr, ws_bytes):
    return int(lib().cqr_backward(m, n, q_ptr, a_ptr, lda, r_ptr, dq_ptr, dr_ptr, da_ptr, stream,
                                  ws_ptr, ws_bytes))


def backward_batched(batch, m, n, q_ptr, a_ptr, lda, stride, r_ptr, dq_ptr, dr_ptr, da_ptr, stream,
                     ws_ptr, ws_bytes):
    return int(lib().cqr_backward_batched(batch, m, n, q_ptr, a_ptr, lda, stride, r_ptr, dq_ptr,
                                          dr_ptr, da_ptr, stream, ws_ptr, ws_bytes))


def plan_batched(ms, ns, bs, schedule: int):
    import numpy as np
    m = np.ascontiguousarray(ms, dtype=np.int64)
    n = np.ascontiguousarray(ns, dtype=np.int64)
    b = None if bs is None else np.ascontiguousarray(bs, dtype=np.int64)
    out = C.c_void_p(0)
    st = lib().cqr_plan_batched(len(m), m.ctypes.data, n.ctypes.data,
                                None if b is None else b.ctypes.data, schedule, C.byref(out))
    check(st, "cqr_plan_batched")
    return out.value


def factor_batched(plan, a_ptrs, lda_ptr, q_ptrs, r_ptrs, info_ptr, stream):
    return int(lib().cqr_factor_batched(plan, a_ptrs, lda_ptr, q_ptrs, r_ptrs, info_ptr, stream))


def plan_destroy(plan) -> None:
    if plan:
        lib().cqr_plan_destroy(plan)


def get_info(stream) -> int:
    v = C.c_int(0)
    check(lib().cqr_get_info(stream, C.byref(v)), "cqr_get_info")
    return v.value


def profile_enable(on: bool) -> None:
    check(lib().cqr_profile_enable(1 if on else 0), "cqr_profile_enable")


def profile_select(kinds=None) -> None:
    """Bracket only these kernel classes (names of KERNEL_KINDS; None = all)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << KERNEL_KINDS.index(k) for k in kinds)
    check(lib().cqr_profile_select(mask), "cqr_profile_select")


def profile_reset() -> None:
    check(lib().cqr_profile_reset(), "cqr_profile_reset")


def profile_query(kind: str) -> dict:
    n = C.c_int64(0)
    ms, fl, by = C.c_double(0), C.c_double(0), C.c_double(0)
    check(lib().cqr_profile_query(KERNEL_KINDS.index(kind), C.byref(n), C.byref(ms), C.byref(fl),
                                  C.byref(by)), "cqr_profile_query")
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}
