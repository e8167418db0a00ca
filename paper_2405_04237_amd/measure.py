"""Accuracy measurement of a factorisation on the device (reporting only).

The quantities are the paper's accuracy measures (section "Testing
environment"): ||Q^T Q - I||_F (also divided by sqrt(n)) and ||QR - A||_F /
||A||_F. They are computed with torch's own FP64 matrix products, which
share nothing with libcqr's kernels, over 4096-row chunks whose results are
added in a fixed pairwise tree, so that the measurement floor (~u sqrt(n))
stays far below the 1e-13 bound being checked at m = 2^22.
"""
from __future__ import annotations

import math

CHUNK = 4096
GROUP = 16  # chunks per batched product


def _pairwise(parts):
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def _xtx_chunks(q):
    """List of per-chunk Q_c^T Q_c (each n x n), in row order."""
    import torch
    m, n = q.shape
    out = []
    full = m // CHUNK * CHUNK
    for s in range(0, full, CHUNK * GROUP):
        e = min(full, s + CHUNK * GROUP)
        k = (e - s) // CHUNK
        blk = q[s:e].reshape(k, CHUNK, n) if q.is_contiguous() else q[s:e].contiguous().reshape(k, CHUNK, n)
        bt = blk.transpose(1, 2).contiguous()
        g = torch.bmm(bt, blk.contiguous())
        out.extend(g.unbind(0))
    if full < m:
        tail = q[full:]
        out.append(tail.t().contiguous() @ tail.contiguous())
    return out


def orthogonality(q, normalised: bool = False) -> float:
    import torch
    n = q.shape[1]
    g = _pairwise(_xtx_chunks(q))
    g = g - torch.eye(n, dtype=g.dtype, device=g.device)
    v = float(torch.linalg.norm(g))
    return v / math.sqrt(n) if normalised else v


def residual(a, q, r) -> float:
    """||A - Q R||_F / ||A||_F, summed per chunk with math.fsum on the host."""
    m = a.shape[0]
    num, den = [], []
    step = CHUNK * GROUP
    for s in range(0, m, step):
        ac = a[s:s + step]
        d = ac - q[s:s + step] @ r
        num.append(float((d * d).sum()))
        den.append(float((ac * ac).sum()))
    return math.sqrt(math.fsum(num)) / math.sqrt(math.fsum(den))
