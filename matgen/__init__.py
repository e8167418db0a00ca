"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the factorisation itself: it only draws
random numbers and builds test matrices with a prescribed spectrum, the way
the paper's test-matrix suite does (section "Testing environment", subsection
"Test matrix suite"): A = U diag(sigma) V^T with U, V orthonormal factors of
random Gaussian matrices and sigma log-spaced so that kappa(A) ~ kappa.

Conventions
-----------
* Every matrix is returned column-major (Fortran order), FP64.
* sigma_i = kappa ** (-(i) / (n - 1)), i = 0..n-1 (descending from 1 to
  1/kappa); the paper writes the same geometric sequence ascending from 1 to
  sigma, which only rescales A.
* U is the Householder Q factor of an m x n N(0,1) matrix, V the Q factor of
  an n x n N(0,1) matrix, each sign-normalised so that the R factor of the
  generating QR has a positive diagonal (which makes Q Haar-distributed).
* Seeds: numpy.random.SeedSequence([2405, 4237, *key]) spawns one child
  generator (PCG64) for U and one for V.

The device generator (``test_matrix_device``) follows the same recipe with
torch's device RNG and torch's Householder QR; it exists because the host
Householder QR of a 2^22 x 1024 Gaussian takes minutes. Its random stream
differs from the host one, so its matrices are a different draw of the same
distribution.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = (2405, 4237)


def seed_sequence(*key: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([*SEED_BASE, *[int(k) for k in key]])


def log_spectrum(n: int, kappa: float) -> np.ndarray:
    """Singular values 1 = s_0 >= ... >= s_{n-1} = 1/kappa, log-spaced."""
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return np.power(float(kappa), -i / (n - 1))


def _haar_columns(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g)  # LAPACK dgeqrf + dorgqr (Householder)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def test_matrix(m: int, n: int, kappa: float, seed: int) -> np.ndarray:
    """A = U diag(sigma) V^T, m x n, column-major FP64, host memory."""
    if m < n or n < 1:
        raise ValueError("need m >= n >= 1")
    ss = seed_sequence(seed, m, n)
    ru, rv = [np.random.default_rng(s) for s in ss.spawn(2)]
    u = _haar_columns(ru, m, n)
    v = _haar_columns(rv, n, n)
    a = (u * log_spectrum(n, kappa)) @ v.T
    return np.asfortranarray(a)


def gaussian_device(m: int, n: int, seed: int, device="cuda", ld: int | None = None):
    """Column-major m x n matrix of i.i.d. N(0,1) entries from torch's device
    RNG (no factorisation involved); well conditioned for m >> n. Stored
    with leading dimension ld (default m)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed_sequence(seed, m, n, 7).generate_state(1, np.uint64)[0]) & ((1 << 63) - 1))
    x = torch.randn((n, m), dtype=torch.float64, device=device, generator=gen).t()
    if ld is None or ld == m:
        return x
    out = torch.empty((n, ld), dtype=torch.float64, device=device).t()[:m]
    out.copy_(x)
    return out


def test_matrix_device(m: int, n: int, kappa: float, seed: int, device="cuda",
                       chunk_rows: int = 1 << 16, ld: int | None = None):
    """Same recipe on a torch device; returns a column-major (m, n) view.

    U is built as the Q factor of an m x n Gaussian through a two-level
    Householder TSQR (chunks of ``chunk_rows`` rows, then the stacked R
    factors), which yields the same Q as one Householder QR of the whole
    Gaussian (the thin Q with positive-diagonal R is unique) while bounding
    the QR workspace. The result is stored with stride (1, ld), ld = m by
    default.
    """
    import torch

    if m < n or n < 1:
        raise ValueError("need m >= n >= 1")
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed_sequence(seed, m, n).generate_state(1, np.uint64)[0]) & ((1 << 63) - 1))
    f64 = torch.float64
    # V on the host with numpy (n x n, cheap), same recipe
    rv = np.random.default_rng(seed_sequence(seed, m, n, 1))
    v = torch.from_numpy(_haar_columns(rv, n, n)).to(device)
    sig = torch.from_numpy(log_spectrum(n, kappa)).to(device)

    ld = m if ld is None else ld
    if ld < m:
        raise ValueError("need ld >= m")
    out = torch.empty((n, ld), dtype=f64, device=device).t()[:m]  # column-major m x n
    nch = max(1, math.ceil(m / chunk_rows))
    if nch == 1 or m <= chunk_rows:
        g = torch.randn((m, n), dtype=f64, device=device, generator=gen)
        q, r = torch.linalg.qr(g)
        d = torch.sign(torch.diagonal(r))
        d[d == 0] = 1
        u = q * d
        out.copy_((u * sig) @ v.T)
        return out
    # level 1: per-chunk Householder QR; keep Q_c in `out`'s storage transiently
    bounds = [(c * chunk_rows, min(m, (c + 1) * chunk_rows)) for c in range(nch)]
    rs = []
    for lo, hi in bounds:
        g = torch.randn((hi - lo, n), dtype=f64, device=device, generator=gen)
        if hi - lo < n:
            raise ValueError("chunk smaller than n")
        q, r = torch.linalg.qr(g)
        out[lo:hi].copy_(q)
        rs.append(r)
        del g, q
    # level 2: QR of the stacked R factors
    q2, r2 = torch.linalg.qr(torch.cat(rs, dim=0))
    d = torch.sign(torch.diagonal(r2))
    d[d == 0] = 1
    q2 = q2 * d
    m2 = (q2 * sig) @ v.T  # fold Sigma V^T into the level-2 factor
    for c, (lo, hi) in enumerate(bounds):
        blk = m2[c * n:(c + 1) * n]
        out[lo:hi].copy_(out[lo:hi] @ blk)
    return out


def hadamard_exact(m: int, n: int, seed: int, pad_rows: int = 0):
    """Exactly representable A = [H T; 0] with known thin QR (Q = [H; 0], R = T).

    H: first n columns of the Sylvester Hadamard matrix of order m0 = 4^t,
    scaled by 2^-t, so H^T H = I with every partial sum exact. T = D (I + E):
    D diagonal with entries in {1/2, 1, 2}, E strictly upper triangular with
    nonzeros only in rows < n/2 and columns >= n/2 (so E^2 = 0 and T^{-1} =
    (I - E) D^{-1} is exact). All intermediate quantities of a Cholesky-based
    QR of A are short dyadic rationals, so any summation order is exact.
    Returns (A, Q, R) as column-major arrays; A has m0 + pad_rows rows.
    """
    t = round(math.log(m, 4))
    if 4 ** t != m or n > m:
        raise ValueError("m must be a power of 4 with m >= n")
    h = np.ones((1, 1))
    while h.shape[0] < m:
        h = np.block([[h, h], [h, -h]])
    hq = h[:, :n] * 2.0 ** (-t)
    rng = np.random.default_rng(seed_sequence(seed, m, n, 7))
    d = 2.0 ** rng.integers(-1, 2, size=n)
    e = np.zeros((n, n))
    half = n // 2
    if half > 0:
        mask = rng.random((half, n - half)) < 0.5
        vals = rng.choice(np.array([-1.0, -0.5, 0.5, 1.0]), size=(half, n - half))
        e[:half, half:] = vals * mask
    tmat = d[:, None] * (np.eye(n) + e)
    a = hq @ tmat  # exact: entries are short dyadics
    q = hq
    if pad_rows:
        a = np.vstack([a, np.zeros((pad_rows, n))])
        q = np.vstack([q, np.zeros((pad_rows, n))])
    return np.asfortranarray(a), np.asfortranarray(q), np.asfortranarray(tmat)


@dataclass(frozen=True)
class Problem:
    m: int
    n: int
    b: int
    kappa: float
    seed: int


def batch_problems(count: int = 512, seed: int = 4, m_lo: int = 2048,
                   m_hi: int = 65536, n_set=(16, 32, 64, 128), b_cap: int = 32,
                   logk_lo: float = 2.0, logk_hi: float = 14.0) -> list[Problem]:
    """Shapes of the batched workload: m ~ U{m_lo..m_hi}, n ~ U(n_set),
    b = min(ceil(n / 2), b_cap), log10 kappa ~ U[logk_lo, logk_hi], one seed each."""
    rng = np.random.default_rng(seed_sequence(seed, count))
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.choice(np.asarray(n_set), size=count)
    ks = 10.0 ** rng.uniform(logk_lo, logk_hi, size=count)
    return [Problem(int(ms[i]), int(ns[i]), int(min((ns[i] + 1) // 2, b_cap)), float(ks[i]),
                    1000 * seed + i) for i in range(count)]


def cotangents(m: int, n: int, seed: int):
    """Upstream gradients for the adjoint: dQ (m x n) and upper-triangular dR,
    i.i.d. N(0,1), column-major."""
    rng = np.random.default_rng(seed_sequence(seed, m, n, 5))
    dq = np.asfortranarray(rng.standard_normal((m, n)))
    dr = np.asfortranarray(np.triu(rng.standard_normal((n, n))))
    return dq, dr


def unit_direction(m: int, n: int, seed: int) -> np.ndarray:
    """Random direction E with ||E||_F = 1 (finite-difference probes)."""
    rng = np.random.default_rng(seed_sequence(seed, m, n, 9))
    e = rng.standard_normal((m, n))
    return np.asfortranarray(e / np.linalg.norm(e))
