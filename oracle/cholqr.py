"""Oracle algorithms: CholeskyQR, CholeskyQR2, shifted CholeskyQR and
shifted CholeskyQR3, CQRGS, CQR2GS and mCQR2GS.

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain FP64 NumPy/SciPy,
the algorithms' steps in the paper's order, no blocking or fusion beyond
what the algorithms state. Library primitives used as steps: BLAS matrix
products, LAPACK ``dpotrf`` (Cholesky with its breakdown index) and
``dtrsm`` through ``scipy.linalg.solve_triangular``.

Readings of the paper where it is silent:
* Summation over m is chunked: every Gram matrix and every projection is the
  sum of per-chunk products over CHUNK-row blocks, added in a fixed pairwise
  tree. The paper is silent on accumulation order; this bounds the rounding
  depth at m = 2^22 the same way the parallel algorithm's per-rank partial
  sums do (section "CholeskyQR", Algorithm 2; Algorithm 8).
* A Cholesky breakdown (non-positive or NaN pivot) raises ``Breakdown`` with
  the 1-based global column of the failing pivot; the paper only says the
  algorithm fails there (sections "CholeskyQR" and "CholeskyQR2").
* The second CQRGS pass of CQR2GS uses the same panel width as the first.
* mCQR2GS (Algorithm 9) leaves R implicit; R is assembled as derived in
  ``mcqr2gs``.
* The run-time choice of CholeskyQR repetitions (section "Conclusion",
  future work) is read as: leave a repetition out when its input's Gram
  matrix is within a tolerance of I, and the re-orthogonalisation update
  when its coefficients Z are below the tolerance (``mcqr2gs(adaptive=)``).
* Shifted CholeskyQR (Algorithm 4): u is the unit roundoff of IEEE binary64,
  2^-53. ||A||_F^2 is the sum of the squared entries, per CHUNK-row block and
  then over blocks in the pairwise tree (the per-rank sums of section
  "Shifted CholeskyQR3").
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

CHUNK = 4096


class Breakdown(ArithmeticError):
    """Cholesky of a Gram matrix met a pivot that is not > 0 (or is NaN)."""

    def __init__(self, column: int):
        super().__init__(f"Gram matrix not positive definite at column {column}")
        self.column = column


def _pairwise(parts):
    """Fixed pairwise tree sum of a list of equally shaped arrays."""
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def xprod(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """X^T Y summed over CHUNK-row blocks in a pairwise tree.

    The local products and their sum are the Gram / projection steps of the
    parallel algorithms (Algorithm 2 lines computing W_i and the Allreduce;
    Algorithm 8 lines computing W_{p,j}, Y_p and their Allreduce), with row
    chunks standing in for processors.
    """
    m = x.shape[0]
    if m == 0:
        return np.zeros((x.shape[1], y.shape[1]))
    parts = [x[i:i + CHUNK].T @ y[i:i + CHUNK] for i in range(0, m, CHUNK)]
    return _pairwise(parts)


def gram(x: np.ndarray) -> np.ndarray:
    """W = X^T X (Algorithm 1, Gram-matrix step), chunked as in ``xprod``."""
    return xprod(x, x)


def chol_upper(w: np.ndarray, col0: int = 0) -> np.ndarray:
    """Upper Cholesky factor U with W = U^T U (Algorithm 1, Cholesky step).

    Uses LAPACK dpotrf on the upper triangle; a failure raises Breakdown with
    the 1-based global column col0 + info.
    """
    c, info = lapack.dpotrf(np.array(w, order="F", copy=True), lower=0, clean=1)
    if info > 0:
        raise Breakdown(col0 + int(info))
    if info < 0:
        raise ValueError("dpotrf argument error")
    # some LAPACK builds let a NaN pivot through; a pivot that is not > 0
    # (NaN included) is a breakdown at that column
    bad = np.flatnonzero(~(np.diag(c) > 0))
    if bad.size:
        raise Breakdown(col0 + int(bad[0]) + 1)
    return np.triu(c)


def _right_solve_upper(x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """X U^{-1} by triangular solve (Algorithm 1, Q := A R^{-1}, via trsm)."""
    # solve U^T Z = X^T for Z = (X U^{-1})^T
    return sla.solve_triangular(u, x.T, trans="T", lower=False, check_finite=False).T


def cqr(x: np.ndarray, col0: int = 0):
    """CholeskyQR, Algorithm 1 (its parallel form, Algorithm 2): returns Q, R."""
    w = gram(x)
    u = chol_upper(w, col0)
    q = _right_solve_upper(x, u)
    return q, u


def cqr2(x: np.ndarray, col0: int = 0):
    """CholeskyQR2, Algorithm 3: CQR twice, R = R2 R1."""
    q1, r1 = cqr(x, col0)
    q, r2 = cqr(q1, col0)
    return q, r2 @ r1


UNIT_ROUNDOFF = 2.0 ** -53


def frobenius_sq(x: np.ndarray) -> float:
    """||X||_F^2: squares of the entries summed per CHUNK-row block, the block
    sums added in the pairwise tree (section "Shifted CholeskyQR3": each rank
    sums the squares of its rows, rank 0 adds the sums)."""
    m = x.shape[0]
    if m == 0:
        return 0.0
    parts = [np.array(np.sum(x[i:i + CHUNK] * x[i:i + CHUNK])) for i in range(0, m, CHUNK)]
    return float(_pairwise(parts))


def scqr_shift(x: np.ndarray) -> float:
    """The shift s = sqrt(m) u ||X||_F^2 of Algorithm 4."""
    return float(np.sqrt(x.shape[0]) * UNIT_ROUNDOFF * frobenius_sq(x))


def scqr(x: np.ndarray, col0: int = 0):
    """Shifted CholeskyQR, Algorithm 4: G = X^T X, W = G + sI, W = R^T R,
    Q = X R^{-1}. Returns Q, R."""
    g = gram(x)
    s = scqr_shift(x)
    w = g + s * np.eye(g.shape[0])
    r = chol_upper(w, col0)
    q = _right_solve_upper(x, r)
    return q, r


def scqr3(x: np.ndarray):
    """Shifted CholeskyQR3, Algorithm 5: [Q1, R1] = sCQR(X);
    [Q, R2] = CQR2(Q1); R = R2 R1."""
    q1, r1 = scqr(x)
    q, r2 = cqr2(q1)
    return q, r2 @ r1


def _panels(n: int, b: int):
    if b < 1:
        raise ValueError("panel width must be >= 1")
    b = min(b, n)
    return [(s, min(s + b, n)) for s in range(0, n, b)]


def cqrgs(a: np.ndarray, b: int):
    """CholeskyQR with block Gram-Schmidt (Algorithm 6; its distributed form
    is Algorithm 8). Returns Q, R; A is not modified.

    Left to right over the panels: CholeskyQR of the panel (its Gram matrix,
    the Cholesky factor, which becomes the diagonal block of R, and the
    triangular solve for the panel's Q), then one block classical
    Gram-Schmidt step that removes the new Q panel from every column to its
    right and records the coefficients as that block row of R.
    """
    m, n = a.shape
    x = np.array(a, dtype=np.float64, order="F", copy=True)
    r = np.zeros((n, n))
    for (s, e) in _panels(n, b):
        panel = x[:, s:e]
        u = chol_upper(gram(panel), s)
        x[:, s:e] = _right_solve_upper(panel, u)
        r[s:e, s:e] = u
        if e < n:
            coef = xprod(x[:, s:e], x[:, e:])
            x[:, e:] -= x[:, s:e] @ coef
            r[s:e, e:] = coef
    return x, r


def cqr2gs(a: np.ndarray, b: int):
    """CholeskyQR2 with Gram-Schmidt (the paper's CQR2GS), Algorithm 7:
    CQRGS twice with the same panel width, then R = R2 R1."""
    q1, r1 = cqrgs(a, b)
    q, r2 = cqrgs(q1, b)
    return q, r2 @ r1


def _gram_distance(w: np.ndarray) -> float:
    """||W - I||_F of a symmetric W, from its upper triangle."""
    d = np.diag(w) - 1.0
    up = np.triu(w, 1)
    return float(np.sqrt(np.sum(d * d) + 2.0 * np.sum(up * up)))


def _cqr_again(x: np.ndarray, col0: int, tol):
    """The repeated CholeskyQR of a nearly orthonormal X. With tol set it is
    left out (Q = X, U = I) when the Gram matrix of X is within tol of I in
    the Frobenius norm: the repetition could only move the orthogonality
    from ||X^T X - I||_F to O(u)."""
    if tol is not None:
        w = gram(x)
        if _gram_distance(w) <= tol:
            return x.copy(), np.eye(x.shape[1])
    return cqr(x, col0)


def mcqr2gs(a: np.ndarray, b: int, adaptive=None):
    """Modified CholeskyQR2 with Gram-Schmidt (mCQR2GS), Algorithm 9.

    The first panel gets CholeskyQR2. Every later panel first loses its
    component along the previous (already final) panel, through a projection
    of all columns to the right of that panel; it is then factored by
    CholeskyQR (factor Ua), re-orthogonalised once against all finished
    panels (coefficients Z), and factored by CholeskyQR again (factor Ub).
    The projected panel therefore equals Q_{1:j-1} (Z Ua) + Q_j (Ub Ua):
    R_{1:j-1,j} gains Z Ua and R_jj = Ub Ua, while the projection
    coefficients fill the previous panel's block row. The paper does not
    write R for this algorithm; this is the bookkeeping that makes A = Q R
    hold.

    adaptive = tol (the run-time choice of repetitions the paper proposes in
    its conclusion): a repeated CholeskyQR is left out when the Gram matrix
    of its input is within tol of I (``_cqr_again``), and the
    re-orthogonalisation update when ||Z||_F <= tol (Z := 0), which changes
    Q_j's orthogonality to the earlier panels by at most ||Z||_F.
    """
    m, n = a.shape
    x = np.array(a, dtype=np.float64, order="F", copy=True)
    r = np.zeros((n, n))
    pan = _panels(n, b)
    s0, e0 = pan[0]
    if adaptive is None:
        x[:, s0:e0], r[s0:e0, s0:e0] = cqr2(x[:, s0:e0], s0)
    else:
        q1, r1 = cqr(x[:, s0:e0], s0)
        q2, r2 = _cqr_again(q1, s0, adaptive)
        x[:, s0:e0], r[s0:e0, s0:e0] = q2, r2 @ r1
    for jj in range(1, len(pan)):
        ps, pe = pan[jj - 1]
        s, e = pan[jj]
        # project the finished previous panel out of everything to its right
        coef = xprod(x[:, ps:pe], x[:, s:])
        x[:, s:] -= x[:, ps:pe] @ coef
        r[ps:pe, s:] = coef
        # first CholeskyQR of the new panel, then one classical Gram-Schmidt
        # pass against all finished panels, then CholeskyQR again
        qt, ua = cqr(x[:, s:e], s)
        z = xprod(x[:, :s], qt)
        if adaptive is not None and np.linalg.norm(z) <= adaptive:
            z = np.zeros_like(z)
        qt = qt - x[:, :s] @ z
        qj, ub = _cqr_again(qt, s, adaptive)
        x[:, s:e] = qj
        r[:s, s:e] += z @ ua
        r[s:e, s:e] = ub @ ua
    return x, r


def householder_qr(a: np.ndarray):
    """Independent reference: LAPACK Householder QR (dgeqrf/dorgqr) with the
    sign normalisation that makes diag(R) > 0 (thin QR is then unique)."""
    q, r = np.linalg.qr(a)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d, d[:, None] * r


def qr_adjoint(q: np.ndarray, r: np.ndarray, dq=None, dr=None) -> np.ndarray:
    """Reverse-mode derivative of the thin QR map A -> (Q, R), m >= n.

    dA = (dQ + Q copyltu(M)) R^{-T},  M = R dR^T - dQ^T Q,
    copyltu(M) = tril(M) + tril(M, -1)^T (the lower triangle mirrored).
    This is the published QR adjoint for full-column-rank A; the paper does
    not differentiate the factorisation. The lower triangle of dR is ignored;
    a missing cotangent counts as zero.
    """
    m, n = q.shape
    dq = np.zeros((m, n)) if dq is None else np.asarray(dq)
    dr = np.zeros((n, n)) if dr is None else np.triu(np.asarray(dr))
    mm = r @ dr.T - xprod(dq, q)
    c = np.tril(mm) + np.tril(mm, -1).T
    g = dq + q @ c
    # right-multiply by R^{-T}: solve Z R^T = G  <=>  R Z^T = G^T
    return sla.solve_triangular(r, g.T, lower=False, check_finite=False).T
