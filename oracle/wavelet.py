"""Orthonormal Haar wavelet transform and the complex soft-threshold prior.

The paper's classical baseline is a wavelet l1 prior (Table 1,
"FISTA-Wavelet"), and its proximal-operator definition (Sec. 2.2, Eq. 3:
prox_{gamma*lambda*r}(x) = argmin_u gamma*lambda*r(u) + 1/2||x - u||^2)
fixes what the plug-in step computes when r is an l1 norm of orthonormal
wavelet detail coefficients: transform, soft-threshold the detail bands,
inverse transform.

Reading taken where the paper is silent: orthonormal Haar with filters
(1, 1)/sqrt(2) and (1, -1)/sqrt(2), separable along every axis, J levels on
the usual pyramid layout (level j acts on the leading ``n >> j`` entries of
every axis), ``J = min(4, floor(log2 n) - 3)``; complex-modulus soft
threshold ``c * max(0, 1 - tau/|c|)`` (0 stays 0) on every coefficient
outside the coarsest approximation block; ``tau = kappa * sigma``.
"""
from __future__ import annotations

import math

import numpy as np

_S = 1.0 / math.sqrt(2.0)


def default_levels(n: int) -> int:
    return max(1, min(4, int(math.floor(math.log2(n))) - 3))


def _haar_axis(c, axis, m):
    """One analysis step along ``axis`` on the leading m entries."""
    sl = [slice(None)] * c.ndim
    sl_e = list(sl)
    sl_o = list(sl)
    sl_e[axis] = slice(0, m, 2)
    sl_o[axis] = slice(1, m, 2)
    e = c[tuple(sl_e)].copy()
    o = c[tuple(sl_o)].copy()
    lo = list(sl)
    hi = list(sl)
    lo[axis] = slice(0, m // 2)
    hi[axis] = slice(m // 2, m)
    c[tuple(lo)] = (e + o) * _S
    c[tuple(hi)] = (e - o) * _S


def _ihaar_axis(c, axis, m):
    sl = [slice(None)] * c.ndim
    lo = list(sl)
    hi = list(sl)
    lo[axis] = slice(0, m // 2)
    hi[axis] = slice(m // 2, m)
    a = c[tuple(lo)].copy()
    d = c[tuple(hi)].copy()
    ev = list(sl)
    od = list(sl)
    ev[axis] = slice(0, m, 2)
    od[axis] = slice(1, m, 2)
    c[tuple(ev)] = (a + d) * _S
    c[tuple(od)] = (a - d) * _S


def haar_forward(x, levels: int):
    """Multilevel separable orthonormal Haar analysis (pyramid layout)."""
    c = np.array(x, dtype=np.complex128, copy=True)
    shape = c.shape
    for j in range(levels):
        sub = tuple(slice(0, n >> j) for n in shape)
        v = c[sub]
        for ax in range(c.ndim):
            _haar_axis(v, ax, shape[ax] >> j)
        c[sub] = v
    return c


def haar_inverse(c, levels: int):
    x = np.array(c, dtype=np.complex128, copy=True)
    shape = x.shape
    for j in reversed(range(levels)):
        sub = tuple(slice(0, n >> j) for n in shape)
        v = x[sub]
        for ax in reversed(range(x.ndim)):
            _ihaar_axis(v, ax, shape[ax] >> j)
        x[sub] = v
    return x


def soft_threshold(c, tau: float):
    """prox of tau*|.| for complex entries: c * max(0, 1 - tau/|c|)."""
    c = np.asarray(c, dtype=np.complex128)
    mag = np.abs(c)
    fac = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    return c * fac


def detail_mask(shape, levels: int):
    """True on detail coefficients, False on the coarsest approximation."""
    m = np.ones(shape, dtype=bool)
    m[tuple(slice(0, n >> levels) for n in shape)] = False
    return m


def wavelet_denoise(u, tau: float, levels: int | None = None):
    """The plug-in wavelet prior D(u): Haar analysis, soft threshold of the
    detail coefficients at tau, Haar synthesis.  This equals
    prox_g(u) for g(v) = tau * ||detail(H v)||_1 (H orthonormal)."""
    u = np.asarray(u, dtype=np.complex128)
    J = default_levels(min(u.shape)) if levels is None else levels
    for n in u.shape:
        if n % (1 << J):
            raise ValueError("image side must be divisible by 2^levels")
    c = haar_forward(u, J)
    m = detail_mask(u.shape, J)
    c[m] = soft_threshold(c[m], tau)
    return haar_inverse(c, J)


def l1_detail(u, levels: int):
    """g(u)/tau = ||detail(H u)||_1 (the convex function behind the prior)."""
    c = haar_forward(u, levels)
    return float(np.abs(c[detail_mask(c.shape, levels)]).sum())
