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
