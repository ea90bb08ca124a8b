"""Image-quality metrics (Sec. 4.3.1): PSNR and SSIM on magnitude images,
PSNR restricted to the region of interest.

Readings: ROI = phantom support (the paper's "brain region");
``PSNR = 20 log10(max_ROI |x_true| / RMSE_ROI(|x_hat|, |x_true|))``;
SSIM after Wang et al. (2004) with a 7x7 uniform window, K1 = 0.01,
K2 = 0.03, data range = max |x_true|, sample (N-1) covariances, averaged
over window centres whose window lies inside the image.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import uniform_filter


def psnr(x_hat, x_true, roi=None) -> float:
    a = np.abs(np.asarray(x_hat, dtype=np.complex128))
    b = np.abs(np.asarray(x_true, dtype=np.complex128))
    if roi is None:
        roi = np.ones(b.shape, dtype=bool)
    err = a[roi] - b[roi]
    mse = float(np.mean(err * err))
    peak = float(b[roi].max())
    if mse == 0.0:
        return math.inf
    return 10.0 * math.log10(peak * peak / mse)


def ssim(x_hat, x_true, win: int = 7, K1: float = 0.01, K2: float = 0.03) -> float:
    a = np.abs(np.asarray(x_hat, dtype=np.complex128))
    b = np.abs(np.asarray(x_true, dtype=np.complex128))
    rng = float(b.max())
    C1 = (K1 * rng) ** 2
    C2 = (K2 * rng) ** 2
    npx = win ** a.ndim
    cov = npx / (npx - 1.0)
    ua = uniform_filter(a, win)
    ub = uniform_filter(b, win)
    vaa = cov * (uniform_filter(a * a, win) - ua * ua)
    vbb = cov * (uniform_filter(b * b, win) - ub * ub)
    vab = cov * (uniform_filter(a * b, win) - ua * ub)
    s = ((2 * ua * ub + C1) * (2 * vab + C2)) / ((ua * ua + ub * ub + C1) * (vaa + vbb + C2))
    h = (win - 1) // 2
    crop = tuple(slice(h, n - h) for n in s.shape)
    return float(s[crop].mean())
