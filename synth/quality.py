"""Restoration quality of a denoised cube against its clean cube.

These are evaluation metrics, not part of the solver. Both are written
from their definitions:

- MPSNR (eq. (29)): mean over bands of 10 log10(N1 N2 / ||u_k - u_clean_k||^2),
  with peak 1, since intensities are in [0, 1].
- MSSIM (eq. (30)): mean over bands of SSIM(u_k, u_clean_k). SSIM is the
  structural similarity of Wang, Bovik, Sheikh and Simoncelli (IEEE TIP
  2004):
  - local means, variances and covariance are taken under an 11 x 11
    circular Gaussian window (sigma 1.5, weights summing to 1);
  - the index is ((2 mu_x mu_y + C1)(2 s_xy + C2)) /
    ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)) with C1 = (0.01 L)^2,
    C2 = (0.03 L)^2 and dynamic range L = 1;
  - the index map is averaged over the window positions that lie inside the
    image.

Cubes are BSQ arrays of shape (N3, N1, N2).
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import correlate1d

WIN, WIN_SIGMA = 11, 1.5
K1, K2, DYN_RANGE = 0.01, 0.03, 1.0


def gaussian_window_1d(size: int = WIN, sigma: float = WIN_SIGMA) -> np.ndarray:
    """1-D factor of the separable Gaussian window (the 2-D window is its
    outer product and sums to 1)."""
    x = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    return g / g.sum()


def _local_mean(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Gaussian-weighted mean over every window that lies inside the image."""
    h = (len(g) - 1) // 2
    m = correlate1d(correlate1d(img, g, axis=-1, mode="constant"), g, axis=-2, mode="constant")
    return m[..., h:img.shape[-2] - h, h:img.shape[-1] - h]


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM index at every inside window position of 2-D images x, y."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.shape != y.shape or x.ndim != 2:
        raise ValueError("two 2-D images of one shape expected")
    if min(x.shape) < WIN:
        raise ValueError(f"images must be at least {WIN} x {WIN}")
    g = gaussian_window_1d()
    c1, c2 = (K1 * DYN_RANGE) ** 2, (K2 * DYN_RANGE) ** 2
    mx, my = _local_mean(x, g), _local_mean(y, g)
    sxx = _local_mean(x * x, g) - mx * mx
    syy = _local_mean(y * y, g) - my * my
    sxy = _local_mean(x * y, g) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(x: np.ndarray, y: np.ndarray) -> float:
    return float(ssim_map(x, y).mean())


def mssim(u: np.ndarray, u_clean: np.ndarray) -> float:
    """Mean over bands of the SSIM of each band, eq. (30)."""
    u, u_clean = np.asarray(u), np.asarray(u_clean)
    return float(np.mean([ssim(u[k], u_clean[k]) for k in range(u.shape[0])]))


def mpsnr(u: np.ndarray, u_clean: np.ndarray) -> float:
    """Mean over bands of the PSNR with peak 1, eq. (29)."""
    u = np.asarray(u, np.float64)
    u_clean = np.asarray(u_clean, np.float64)
    n3 = u.shape[0]
    err = ((u - u_clean) ** 2).reshape(n3, -1).sum(axis=1)
    return float(np.mean(10.0 * np.log10(u[0].size / err)))
