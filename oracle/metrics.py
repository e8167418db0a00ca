"""Accuracy measures of a computed QR factorisation.

TEST INFRASTRUCTURE ONLY. The paper judges a factorisation by the loss of
orthogonality ||Q^T Q - I||_F / sqrt(n) and the residual ||QR - A||_F /
||A||_F (section "Testing environment"). Both are computed here so that the
measurement floor sits well below the quantities measured: Q^T Q is summed
over 4096-row chunks in a pairwise tree, and the residual squares are summed
per chunk with math.fsum.
"""
from __future__ import annotations

import math

import numpy as np

from .cholqr import xprod

_CH = 4096


def orthogonality(q: np.ndarray, normalised: bool = False) -> float:
    """||Q^T Q - I||_F (divided by sqrt(n) when ``normalised``)."""
    n = q.shape[1]
    g = xprod(q, q)
    g[np.diag_indices(n)] -= 1.0
    v = float(np.linalg.norm(g))
    return v / math.sqrt(n) if normalised else v


def residual(a: np.ndarray, q: np.ndarray, r: np.ndarray) -> float:
    """||A - Q R||_F / ||A||_F."""
    m = a.shape[0]
    num, den = [], []
    for i in range(0, m, _CH):
        ac = a[i:i + _CH]
        d = ac - q[i:i + _CH] @ r
        num.append(float(np.einsum("ij,ij->", d, d)))
        den.append(float(np.einsum("ij,ij->", ac, ac)))
    return math.sqrt(math.fsum(num)) / math.sqrt(math.fsum(den))


def rel_fro(x: np.ndarray, ref: np.ndarray) -> float:
    """||X - ref||_F / ||ref||_F."""
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
