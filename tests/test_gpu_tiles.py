"""Kernel variants of the trailing update and the projection (the tile
shapes the autotuner chooses between): an update with a 64-column slab of Y
in LDS, 64 x 128 (or 64 x 64) register tiles held over the whole inner
dimension, or 32 x 64 tiles; projections with 64 x 128 or 64 x 64 tiles.

Every variant forms each entry from the same MFMA operations in the same
order (the input entry first, then the inner dimension in ascending groups
of four), so Q and R must agree bit for bit across all of them, at every
shape: ragged row counts (a partial last row tile), ragged last panels
(column counts that are not multiples of the tile), strides that rule a
variant out (odd leading dimension: every variant falls back to the same
kernel), panels of 64, 128 and 256 columns, and both schedules. One run per
shape is also held to the oracle's bounds (Algorithms 7 and 9).
"""
import numpy as np
import pytest

import matgen
import oracle
from tests.util import check_r, r_bars, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2405_04237_amd as cqr  # noqa: E402

VARIANTS = [(u, p) for u in ("auto", "slab", "wide", "narrow", "resident")
            for p in ("auto", "wide", "narrow")]


@pytest.mark.parametrize("m,n,b,kappa,ld,sched", [
    (4096, 64, 16, 1e12, None, "mod"),     # the small workload (short updates only)
    (5000, 300, 128, 1e15, None, "mod"),   # m % 64 = 8; last panel 44 columns; q % 8 = 4
    (6001, 272, 96, 1e10, 6007, "mod"),    # odd stride: no vector loads, common fallback
    (65536, 512, 128, 1e15, None, "mod"),  # long updates up to 384 inner columns
    (20000, 600, 256, 1e15, None, "mod"),  # 256-column panels (no LDS slab), last 88 wide
    (70000, 256, 64, 1e12, 70016, "orig"), # CQR2GS: updates of 192..64 columns
])
def test_tile_variants_bitwise_equal(m, n, b, kappa, ld, sched):
    a = matgen.test_matrix(m, n, kappa, seed=71)
    ad = to_dev(a, ld)
    ref = None
    for ut, pt in VARIANTS:
        q, r = cqr.qr(ad, b=b, schedule=sched, update_tile=ut, proj_tile=pt)
        torch.cuda.synchronize()
        if ref is None:
            ref = (q.clone(), r.clone())
            continue
        assert torch.equal(q, ref[0]) and torch.equal(r, ref[1]), (ut, pt)
    q, r = to_host(ref[0]), to_host(ref[1])
    f = oracle.mcqr2gs if sched == "mod" else oracle.cqr2gs
    qo, ro = f(a, b)
    orth = oracle.orthogonality(q)
    if sched == "mod":
        assert orth <= 1e-13
    else:
        assert orth <= max(1e-13, 10 * oracle.orthogonality(qo))
    assert oracle.residual(a, q, r) <= 1e-14
    check_r(r, ro, r_bars(a, ro, kappa), f"tiles {sched} {m}x{n} b={b}")


def test_tile_variant_breakdown_column():
    """A rank-deficient panel is reported at the same column by every variant."""
    a = matgen.test_matrix(9000, 320, 10.0, seed=72)
    a[:, 201] = 0.0
    ad = to_dev(a)
    for ut in ("slab", "wide", "narrow", "resident"):
        with pytest.raises(cqr.Breakdown) as e:
            cqr.qr(ad, b=128, schedule="mod", update_tile=ut)
        assert e.value.column == 202, ut
