"""Independent FP64 Kaiser-Bessel gridding reference and its exact error.

The paper leaves the non-uniform Fourier transform's algorithm open
(Sec. 2.1, Eq. 1).  The GPU library approximates the exact operator of
``oracle.ndft`` by Kaiser-Bessel (KB) gridding with kernel width W = 6 and
oversampling 2.  This module is a second, deliberately plain, FP64
implementation of that approximation (zero-pad + deapodise + numpy FFT +
explicit taps) plus the closed-form per-(pixel, sample) response of any KB
gridding operator.  It is used only to pin the exact NDFT oracle (two
independent computations must agree within the predicted KB error) and to
predict the approximation floor of the GPU operator.  It is never a parity
target for the GPU: parity is always against ``oracle.ndft``.

Definitions (grid units, K = osf*n grid points per axis):
* kernel  phi(u) = I0(beta*sqrt(1 - (2u/W)^2)) for |u| <= W/2, else 0
* its FT  Phi(nu) = W*sinh(z)/z with z = sqrt(beta^2 - (pi*W*nu)^2)
          (W*sin(|z|)/|z| when the radicand is negative)
* Beatty's width rule  beta = pi*sqrt((W/osf)^2*(osf - 1/2)^2 - 0.8)
* grid coordinate of a sample  g = k*K/(2*pi); taps j = floor(g - W/2) + 1
  ... floor(g - W/2) + W (the half-open window (g - W/2, g + W/2]), wrapped
  modulo K.
* pixel r sits at grid index r mod K; the forward uses the FFT with kernel
  exp(-2*pi*i*j*r/K), the adjoint its conjugate.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import i0


def beatty_beta(W: int = 6, osf: float = 2.0) -> float:
    return math.pi * math.sqrt((W / osf) ** 2 * (osf - 0.5) ** 2 - 0.8)


def kb_phi(u, W: int, beta: float):
    u = np.asarray(u, dtype=np.float64)
    t = 1.0 - (2.0 * u / W) ** 2
    out = np.zeros_like(u)
    ok = np.abs(u) <= W / 2
    out[ok] = i0(beta * np.sqrt(np.maximum(t[ok], 0.0)))
    return out


def kb_Phi(nu, W: int, beta: float):
    nu = np.asarray(nu, dtype=np.float64)
    z2 = beta ** 2 - (math.pi * W * nu) ** 2
    out = np.empty_like(nu)
    pos = z2 > 1e-300
    neg = z2 < -1e-300
    zer = ~(pos | neg)
    z = np.sqrt(z2[pos])
    out[pos] = W * np.sinh(z) / z
    zn = np.sqrt(-z2[neg])
    out[neg] = W * np.sin(zn) / zn
    out[zer] = W
    return out


def _r(n):
    return np.arange(n, dtype=np.float64) - n // 2


def _taps(g, W):
    """Tap start index and the W tap offsets for grid coordinates g."""
    j0 = np.floor(g - W / 2.0) + 1.0
    j = j0[..., None] + np.arange(W, dtype=np.float64)
    return j


class KBGridding:
    """FP64 KB-gridding approximation of ``oracle.ndft`` (2D and 3D)."""

    def __init__(self, shape, traj, W: int = 6, osf: int = 2, beta: float | None = None):
        self.shape = tuple(shape)
        self.d = len(shape)
        self.W = W
        self.osf = osf
        self.beta = beatty_beta(W, osf) if beta is None else beta
        self.K = tuple(osf * n for n in shape)
        k = np.asarray(traj, dtype=np.float64)
        self.M = k.shape[0]
        # per axis, in image-axis order (slowest first): traj column d-1-a
        self.idx = []
        self.wts = []
        for a, (n, K) in enumerate(zip(self.shape, self.K)):
            g = k[:, self.d - 1 - a] * K / (2 * math.pi)
            j = _taps(g, W)
            self.wts.append(kb_phi(g[:, None] - j, W, self.beta))
            self.idx.append(np.mod(j, K).astype(np.int64))
        self.deapod = [1.0 / kb_Phi(_r(n) / K, W, self.beta) for n, K in zip(self.shape, self.K)]
        self.scale = 1.0 / math.sqrt(int(np.prod(shape)))

    def _pre(self, img):
        z = img.copy()
        for a, dp in enumerate(self.deapod):
            sh = [1] * self.d
            sh[a] = -1
            z = z * dp.reshape(sh)
        grid = np.zeros(self.K, dtype=np.complex128)
        ix = np.ix_(*[np.mod(_r(n), K).astype(np.int64) for n, K in zip(self.shape, self.K)])
        grid[ix] = z
        return grid

    def _post(self, grid):
        ix = np.ix_(*[np.mod(_r(n), K).astype(np.int64) for n, K in zip(self.shape, self.K)])
        z = grid[ix]
        for a, dp in enumerate(self.deapod):
            sh = [1] * self.d
            sh[a] = -1
            z = z * dp.reshape(sh)
        return z

    def _interp(self, G):
        y = np.zeros(self.M, dtype=np.complex128)
        W = self.W
        if self.d == 2:
            for a in range(W):
                for b in range(W):
                    y += self.wts[0][:, a] * self.wts[1][:, b] * G[self.idx[0][:, a], self.idx[1][:, b]]
        else:
            for a in range(W):
                for b in range(W):
                    for c in range(W):
                        y += (self.wts[0][:, a] * self.wts[1][:, b] * self.wts[2][:, c]
                              * G[self.idx[0][:, a], self.idx[1][:, b], self.idx[2][:, c]])
        return y

    def _spread(self, v):
        # H[j] = sum over samples and taps landing on j of weight * v (bincount
        # accumulates the same sums as an explicit loop over taps)
        G = int(np.prod(self.K))
        re = np.zeros(G)
        im = np.zeros(G)
        W = self.W
        if self.d == 2:
            for a in range(W):
                for b in range(W):
                    flat = self.idx[0][:, a] * self.K[1] + self.idx[1][:, b]
                    c = self.wts[0][:, a] * self.wts[1][:, b] * v
                    re += np.bincount(flat, c.real, G)
                    im += np.bincount(flat, c.imag, G)
        else:
            for a in range(W):
                for b in range(W):
                    for cc in range(W):
                        flat = ((self.idx[0][:, a] * self.K[1] + self.idx[1][:, b]) * self.K[2]
                                + self.idx[2][:, cc])
                        c = self.wts[0][:, a] * self.wts[1][:, b] * self.wts[2][:, cc] * v
                        re += np.bincount(flat, c.real, G)
                        im += np.bincount(flat, c.imag, G)
        return (re + 1j * im).reshape(self.K)

    def forward(self, x, smaps):
        x = np.asarray(x, dtype=np.complex128)
        S = np.asarray(smaps, dtype=np.complex128)
        y = np.empty((S.shape[0], self.M), dtype=np.complex128)
        for l in range(S.shape[0]):
            G = np.fft.fftn(self._pre(S[l] * x))
            y[l] = self._interp(G) * self.scale
        return y

    def adjoint(self, y, smaps, dcf=None):
        y = np.asarray(y, dtype=np.complex128)
        S = np.asarray(smaps, dtype=np.complex128)
        w = np.ones(self.M) if dcf is None else np.asarray(dcf, dtype=np.float64)
        out = np.zeros(self.shape, dtype=np.complex128)
        Gtot = int(np.prod(self.K))
        for l in range(S.shape[0]):
            H = self._spread(w * y[l])
            # unnormalised inverse DFT (kernel exp(+2 pi i j r / K))
            z = self._post(np.fft.ifftn(H) * Gtot)
            out += np.conj(S[l]) * z
        return out * self.scale

    def normal(self, x, smaps, dcf=None):
        return self.adjoint(self.forward(x, smaps), smaps, dcf)


def response_1d(r, g, K: int, W: int = 6, beta: float | None = None):
    """Exact gridded response of pixel r at grid coordinate g, divided by
    the exact exponential: ``sum_taps phi(g-j) exp(-2 pi i (j-g) r/K) / Phi(r/K)``.
    Equals 1 for an error-free gridding; |value - 1| is the alias error of
    this (pixel, sample) pair.  Broadcasts over r and g."""
    beta = beatty_beta(W, 2) if beta is None else beta
    r = np.asarray(r, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    j = _taps(g, W)
    ph = kb_phi(g[..., None] - j, W, beta)
    e = np.exp(-2j * math.pi * (j - g[..., None]) * r[..., None] / K)
    return (ph * e).sum(-1) / kb_Phi(r / K, W, beta)


def response_poisson_1d(r: float, g: float, K: int, W: int = 6, beta: float | None = None,
                        P: int = 200000):
    """The same response by Poisson summation:
    ``1 + sum_{p != 0} Phi(r/K + p)/Phi(r/K) * exp(-2 pi i g p)`` truncated at
    |p| <= P (the terms decay like 1/p, so the tail is O(1e-6/P))."""
    beta = beatty_beta(W, 2) if beta is None else beta
    p = np.arange(-P, P + 1, dtype=np.float64)
    p = p[p != 0]
    terms = kb_Phi(r / K + p, W, beta) * np.exp(-2j * math.pi * g * p)
    return 1.0 + terms.sum() / kb_Phi(np.array([r / K]), W, beta)[0]


def predicted_rel_rms_white(n: int, d: int = 2, osf: int = 2, W: int = 6, n_g: int = 512,
                            beta: float | None = None) -> float:
    """Predicted relative RMS error of a KB-gridded forward operator applied
    to white (i.i.d.) input, averaged over grid positions g uniform in one
    cell: ``sqrt(E_g mean_r |prod_a R(r_a, g_a) - 1|^2)`` for a separable
    kernel.  Computed from the exact 1D responses by Monte-Carlo-free
    quadrature over g in [0, 1)^d (midpoint rule, n_g points per axis)."""
    K = osf * n
    beta = beatty_beta(W, osf) if beta is None else beta
    r = _r(n)
    g = (np.arange(n_g) + 0.5) / n_g
    R = response_1d(r[None, :], g[:, None], K, W, beta)        # [n_g, n]
    if d == 2:
        # E over (gx, gy) and (rx, ry) of |Rx Ry - 1|^2 with independent axes
        m2 = (np.abs(R) ** 2).mean()
        m1 = R.mean()
        e = m2 * m2 - 2 * (m1 * m1).real + 1.0
    elif d == 3:
        m2 = (np.abs(R) ** 2).mean()
        m1 = R.mean()
        e = m2 ** 3 - 2 * (m1 ** 3).real + 1.0
    else:
        e = (np.abs(R - 1) ** 2).mean()
    return float(math.sqrt(max(e, 0.0)))
