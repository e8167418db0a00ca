"""Why the batched workload's default panel width is min(ceil(n/2), 32)
rather than min(n, 32): with n <= 32 the latter is a single panel, i.e.
CholeskyQR2 (Algorithm 3), which the paper finds unstable beyond kappa of
about 1e8 (section "CholeskyQR2"). On matrices of the workload's recipe with
n <= 32 and kappa well past that limit, the oracle's single-panel run breaks
down or misses the orthogonality bound, while two panels of ceil(n/2)
columns (mCQR2GS, Algorithm 9) meet the bounds. Oracle only (CPU)."""
import pytest

import matgen
import oracle

# (m, n, kappa): shapes and condition numbers inside the batched workload's
# ranges (m in [2048, 65536], n in {16, 32}, log10 kappa in [2, 14])
CASES = [(2048, 16, 1e12), (4096, 32, 1e11), (6000, 16, 1e14), (3000, 32, 1e13)]


@pytest.mark.parametrize("m,n,kappa", CASES)
def test_single_panel_fails_two_panels_hold(m, n, kappa):
    a = matgen.test_matrix(m, n, kappa, seed=77)
    try:
        q, r = oracle.mcqr2gs(a, n)  # b = min(n, 32) = n: one panel
        failed = oracle.orthogonality(q) > 1e-13 or oracle.residual(a, q, r) > 1e-14
    except oracle.Breakdown:
        failed = True
    assert failed, "CholeskyQR2 alone was expected to fail past kappa = 1e8"
    q, r = oracle.mcqr2gs(a, (n + 1) // 2)
    assert oracle.orthogonality(q) <= 1e-13
    assert oracle.residual(a, q, r) <= 1e-14


def test_workload_default_panel_is_two_or_more_panels():
    for p in matgen.batch_problems():
        assert p.b == min((p.n + 1) // 2, 32)
        assert (p.n + p.b - 1) // p.b >= 2
