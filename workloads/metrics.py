"""Image-quality scores used in Sec. 6 of the paper.

Both work on luminance in [0, 1]: level k of L maps to k/(L-1) (for the binary case
-1/+1 maps to 0/1).
* PSNR = 20 log10(max(x) / sqrt(MSE(x, y))) with the peak the maximum of the original.
* SSIM: the single-window formula the paper prints (sample means, variances and
  covariance over the whole image) and the usual windowed form (Gaussian window of
  standard deviation 1.5 truncated at 11x11, K1 = 0.01, K2 = 0.03, dynamic range 1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import gaussian_filter


def psnr(x: np.ndarray, y: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mse = float(np.mean((x - y) ** 2))
    peak = float(x.max())
    if mse == 0.0:
        return math.inf
    return 20.0 * math.log10(peak / math.sqrt(mse))


def _consts(dynamic_range: float):
    return (0.01 * dynamic_range) ** 2, (0.03 * dynamic_range) ** 2


def ssim_global(x: np.ndarray, y: np.ndarray, dynamic_range: float = 1.0) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    c1, c2 = _consts(dynamic_range)
    mx, my = x.mean(), y.mean()
    vx, vy = x.var(ddof=1), y.var(ddof=1)
    cxy = ((x - mx) * (y - my)).sum() / (x.size - 1)
    return float(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx ** 2 + my ** 2 + c1) * (vx + vy + c2)))


def ssim_windowed(x: np.ndarray, y: np.ndarray, dynamic_range: float = 1.0, sigma: float = 1.5) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    c1, c2 = _consts(dynamic_range)
    f = lambda a: gaussian_filter(a, sigma=sigma, truncate=3.5, mode="reflect")  # noqa: E731
    mx, my = f(x), f(y)
    sxx = f(x * x) - mx * mx
    syy = f(y * y) - my * my
    sxy = f(x * y) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(s.mean())


def luminance_levels(levels: np.ndarray, L: int) -> np.ndarray:
    return np.asarray(levels, dtype=np.float64) / (L - 1)


def luminance_values(values: np.ndarray, vmin: float, vmax: float) -> np.ndarray:
    return (np.asarray(values, dtype=np.float64) - vmin) / (vmax - vmin)
