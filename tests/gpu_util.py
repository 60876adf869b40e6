"""Helpers shared by the GPU parity tests (host-side comparison only)."""
import numpy as np


def to_device_colmajor(A: np.ndarray, lda: int | None = None, fill: float = np.nan):
    """Copy host matrix A into a column-major CUDA tensor with leading
    dimension lda (rows beyond A's are filled with `fill`)."""
    import torch

    m, n = A.shape
    lda = m if lda is None else lda
    buf = np.full((n, lda), fill, dtype=np.float64)  # row-major (n x lda) = col-major (lda x n)
    buf[:, :m] = A.T
    t = torch.from_numpy(buf).cuda()
    return t.T[:m, :] if lda == m else t.T, lda


def from_device(t, m):
    return t.T.contiguous().cpu().numpy().T[:m, :] if t.shape[0] != m else t.cpu().numpy()


def sy_compare(Aout_gpu: np.ndarray, tau_gpu: np.ndarray, Aout_orc: np.ndarray, tau_orc: np.ndarray,
               w: int, ncols: int | None = None):
    """Max differences of band entries, stored reflectors and tau (columns < ncols)."""
    n = Aout_orc.shape[0]
    nc = n if ncols is None else ncols
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    band = (i - j >= 0) & (i - j <= w) & (j < nc)
    refl = (i - j > w) & (j < nc)
    d_band = float(np.max(np.abs(Aout_gpu[band] - Aout_orc[band]))) if band.any() else 0.0
    d_refl = float(np.max(np.abs(Aout_gpu[refl] - Aout_orc[refl]))) if refl.any() else 0.0
    k = min(nc, len(tau_orc))
    d_tau = float(np.max(np.abs(tau_gpu[:k] - tau_orc[:k]))) if k > 0 else 0.0
    return d_band, d_refl, d_tau


def ge_compare(Ag, tqg, tpg, Ao, tqo, tpo, w, nsteps=None):
    m, n = Ao.shape
    ns = n if nsteps is None else nsteps
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    band = (j - i >= 0) & (j - i <= w) & (i < ns)
    left = (i > j) & (j < ns)
    right = (j - i > w) & (i < ns)
    f = lambda msk: float(np.max(np.abs(Ag[msk] - Ao[msk]))) if msk.any() else 0.0
    return (f(band), f(left), f(right), float(np.max(np.abs(tqg[:ns] - tqo[:ns]), initial=0.0)),
            float(np.max(np.abs(tpg[:ns] - tpo[:ns]), initial=0.0)))


def sy_band_max(Ao: np.ndarray, w: int, ncols: int | None = None) -> float:
    """Largest |entry| of the symmetric band (0 <= i-j <= w) of a reduced
    matrix: the scale of the band-entry tolerance (each entry of a backward
    stable reduction is accurate to about u n times the largest one)."""
    n = Ao.shape[0]
    nc = n if ncols is None else ncols
    i = np.arange(n)[:, None]
    j = np.arange(nc)[None, :]
    band = (i - j >= 0) & (i - j <= w)
    return float(np.abs(Ao[:, :nc][band]).max())


def ge_band_max(Ao: np.ndarray, w: int, lower: int = 0) -> float:
    """Largest |entry| of the band -lower <= j-i <= w of a reduced matrix."""
    m, n = Ao.shape
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    band = (j - i >= -lower) & (j - i <= w)
    return float(np.abs(Ao[band]).max())
