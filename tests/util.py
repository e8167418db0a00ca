"""Host <-> device helpers for the GPU tests (column-major FP64 layout)."""
import numpy as np

U = 2.0 ** -53


def to_dev(a: np.ndarray, ld: int | None = None):
    """Column-major device copy of a host matrix, optionally with padded ld."""
    import torch
    m, n = a.shape
    ld = m if ld is None else ld
    host = np.zeros((n, ld))
    host[:, :m] = np.asarray(a).T
    return torch.from_numpy(host).to("cuda").t()[:m]


def to_host(t) -> np.ndarray:
    return np.asfortranarray(t.detach().cpu().numpy())


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def r_bars(a: np.ndarray, r_oracle: np.ndarray, kappa: float, r_householder=None):
    """Tolerances for a computed R against the oracle's R.

    * ``first_order``: 100 n u kappa, relative Frobenius (a first-order
      perturbation of the unique R under backward errors of size c n u per
      column). Vacuous for kappa >~ 1e12 at these n.
    * ``spread``: 10 x the distance between the oracle's R and LAPACK's
      Householder R (an independent backward-stable algorithm, sign
      normalised). Two backward-stable QR algorithms land within rounding
      noise of each other; a third one (the GPU) must not be farther from the
      oracle than ten times that spread (triangle inequality, with margin).
      Meaningful at every kappa. It never falls below max(4, n) units of
      roundoff: the two references may agree more closely with each other
      than with a third summation order (the batched kernel sums hundreds of
      rows sequentially per accumulator; n = 1 is a single rounded norm),
      and an R computed in any order carries rounding of about that size.
    * ``elementwise``: where 100 n u kappa < 1e-6, the same first-order bound
      on max |dR_ij| relative to max |R_ij|; None above.
    """
    import oracle
    n = a.shape[1]
    rh = oracle.householder_qr(a)[1] if r_householder is None else r_householder
    fo = 100 * n * U * kappa
    spread = oracle.rel_fro(r_oracle, rh)
    return {"first_order": fo, "spread": max(10 * spread, max(4, n) * U),
            "observed_spread": spread, "elementwise": fo if fo < 1e-6 else None}


def check_r(r: np.ndarray, r_oracle: np.ndarray, bars: dict, label: str = "") -> float:
    """Assert R against the oracle's R under ``bars`` (see r_bars); returns
    the observed relative Frobenius difference (printed for the record)."""
    import oracle
    d = oracle.rel_fro(r, r_oracle)
    print(f"{label} |R - R_oracle|_F / |R_oracle|_F = {d:.3e} "
          f"(oracle vs Householder {bars['observed_spread']:.3e})")
    assert d <= bars["first_order"], (label, d, bars)
    assert d <= bars["spread"], (label, d, bars)
    if bars["elementwise"] is not None:
        el = float(np.max(np.abs(r - r_oracle)) / np.max(np.abs(r_oracle)))
        assert el <= bars["elementwise"], (label, el, bars)
    return d
