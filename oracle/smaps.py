"""FP64 reference of the coil sensitivity estimate from the k-space centre.
Test infrastructure: only the tests, the smoke check and the benchmark's
CPU baseline use it.

Sec. 4.1 estimates the maps S_l from the centre of k-space (a 20 x 20
Hamming window), brings them to the image domain and masks them to the
anatomy.  Read for non-Cartesian data as:

* window: each sample m is weighted by h(kx) h(ky) [h(kz)], with the
  frequency in grid units kappa = k * n / (2 pi) of its axis and
  h(kappa) = 0.54 + 0.46 cos(pi kappa / c) for |kappa| <= c, 0 beyond, the
  half-width c = width / 2 (= 10 for the 20 x 20 window); the density
  weights, when given, multiply in;
* low-resolution coil images z_l = F^H (w h y_l) (the adjoint with unit maps,
  one coil at a time);
* root-sum-of-squares normalisation s = sqrt(sum_l |z_l|^2), S_l = z_l / s;
* mask: S_l = 0 where s <= threshold * max s (threshold 0: no mask).
"""
from __future__ import annotations

import numpy as np

from . import ndft


def hamming(kappa, half_width: float):
    """h(kappa) = 0.54 + 0.46 cos(pi kappa / c) on |kappa| <= c, else 0."""
    kappa = np.asarray(kappa, dtype=np.float64)
    h = 0.54 + 0.46 * np.cos(np.pi * kappa / half_width)
    return np.where(np.abs(kappa) <= half_width, h, 0.0)


def window_weights(traj, shape, width: float = 20.0, dcf=None):
    """Per-sample weights dcf[m] * prod_axis h(kappa_axis) (shape slowest-first,
    trajectory columns ordered x, y[, z])."""
    traj = np.asarray(traj, dtype=np.float64)
    d = traj.shape[1]
    sizes = list(shape)[::-1]            # n_x, n_y[, n_z]
    w = np.ones(traj.shape[0])
    for a in range(d):
        w = w * hamming(traj[:, a] * sizes[a] / (2.0 * np.pi), width / 2.0)
    if dcf is not None:
        w = w * np.asarray(dcf, dtype=np.float64)
    return w


def coil_images(y, traj, shape, width: float = 20.0, dcf=None):
    """z_l = F^H (window * dcf * y_l), one coil at a time; [L][shape]."""
    y = np.asarray(y)
    w = window_weights(traj, shape, width, dcf)
    ones = np.ones((1,) + tuple(shape), dtype=np.complex128)
    return np.stack([ndft.adjoint(y[l:l + 1], ones, traj, w) for l in range(y.shape[0])])


def estimate(y, traj, shape, width: float = 20.0, dcf=None, threshold: float = 0.05):
    """Sensitivity maps [L][shape] and the mask (boolean [shape])."""
    z = coil_images(y, traj, shape, width, dcf)
    s = np.sqrt(np.sum(np.abs(z) ** 2, axis=0))
    mask = s > threshold * s.max() if threshold > 0 else np.ones(s.shape, dtype=bool)
    S = np.where(mask, z / np.where(s > 0, s, 1.0), 0.0)
    return S, mask
