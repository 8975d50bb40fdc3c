"""FP64 SSIM -- TEST INFRASTRUCTURE (the quality index the paper reports beside PSNR, Sec. III-B,
Tables 1 and 2, citing Wang, Bovik, Sheikh and Simoncelli).

Definition used (the reference formulation of that index):
  * an 11 x 11 Gaussian window with standard deviation 1.5, normalised to sum 1;
  * at every position where the window lies inside the image ('valid' region, (H-10) x (W-10)):
      mu_x = sum w x,  sigma_x^2 = sum w x^2 - mu_x^2,  sigma_xy = sum w x y - mu_x mu_y  (same for y);
      SSIM = ((2 mu_x mu_y + C1)(2 sigma_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
      C1 = (0.01 peak)^2, C2 = (0.03 peak)^2;
  * the index is the mean over the valid positions.
Plain NumPy over explicit window views; it shares no code with the HIP library.
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

WIN = 11
SIGMA = 1.5
K1, K2 = 0.01, 0.03


def gaussian_window() -> np.ndarray:
    i = np.arange(WIN) - (WIN - 1) / 2.0
    g = np.exp(-(i * i) / (2.0 * SIGMA * SIGMA))
    w = np.outer(g, g)
    return w / w.sum()


def ssim_map(x, y, peak: float = 255.0) -> np.ndarray:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.shape != y.shape or min(x.shape) < WIN:
        raise ValueError("images must have the same shape, at least 11 x 11")
    w = gaussian_window()
    def wsum(a):
        return np.einsum("ijkl,kl->ij", sliding_window_view(a, (WIN, WIN)), w)
    mx, my = wsum(x), wsum(y)
    sxx = wsum(x * x) - mx * mx
    syy = wsum(y * y) - my * my
    sxy = wsum(x * y) - mx * my
    c1, c2 = (K1 * peak) ** 2, (K2 * peak) ** 2
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(x, y, peak: float = 255.0) -> float:
    return float(np.mean(ssim_map(x, y, peak)))
