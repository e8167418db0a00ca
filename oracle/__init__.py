"""Oracle for CholeskyQR2 with block Gram-Schmidt (arXiv 2405.04237).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow FP64 CPU
implementation used to check the GPU library. Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does. It shares no code with the GPU library.
"""
from .cholqr import (Breakdown, gram, xprod, chol_upper, cqr, cqr2, cqrgs, cqr2gs,
                  mcqr2gs, qr_adjoint, householder_qr, frobenius_sq, scqr_shift, scqr,
                  scqr3, UNIT_ROUNDOFF)
from .metrics import orthogonality, residual, rel_fro

__all__ = ["Breakdown", "gram", "xprod", "chol_upper", "cqr", "cqr2", "cqrgs",
           "cqr2gs", "mcqr2gs", "qr_adjoint", "householder_qr", "orthogonality",
           "residual", "rel_fro", "frobenius_sq", "scqr_shift", "scqr", "scqr3",
           "UNIT_ROUNDOFF"]
