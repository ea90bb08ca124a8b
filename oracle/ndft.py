"""Exact multicoil non-uniform discrete Fourier operator (FP64).

Follows the multicoil forward model of Sec. 2.1, Eq. 1: coil l measures
``y_l = F_Omega S_l x``.  The paper leaves F_Omega's convention open; the
reading taken here is
* sign ``exp(-i <k_m, r>)`` in the forward direction,
* r the centred integer pixel coordinates ``i - n/2`` along every axis,
* k in radians per pixel (trajectory ``[M][d]`` ordered ``(kx, ky[, kz])``),
* orthonormal scale ``N^{-1/2}`` so that Parseval holds and, for coil maps
  with unit sum of squares under full Cartesian sampling, ``A^H A = I``.

The adjoint applies the density-compensation weighting D_w of the weighted
data term ``f_w(x) = 1/2 sum_l ||D_w^{1/2}(F S_l x - y_l)||^2`` (the DCF
used as a k-space weighting); ``w = None`` means D_w = I.

The sum over pixels is computed exactly by separable factorisation:
``exp(-i<k, r>) = prod_axis exp(-i k_axis r_axis)``, which turns each coil's
sum into a dense matrix product followed by a row-wise dot (no
approximation, no FFT, no gridding).
"""
from __future__ import annotations

import numpy as np

_CHUNK = 8192  # samples per block in 3D to bound memory


def _r(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - n // 2


def _as(x, dt):
    return np.asarray(x).astype(dt, copy=False)


def forward(x, smaps, traj):
    """A x: ``y[l, m] = N^{-1/2} sum_r S_l[r] x[r] exp(-i <k_m, r>)``.

    x: ``[ny][nx]`` or ``[nz][ny][nx]``; smaps: ``[L][...]``; traj ``[M][d]``.
    Returns complex128 ``[L][M]``.
    """
    x = _as(x, np.complex128)
    S = _as(smaps, np.complex128)
    k = _as(traj, np.float64)
    d = x.ndim
    N = x.size
    L = S.shape[0]
    M = k.shape[0]
    scale = 1.0 / np.sqrt(N)
    y = np.empty((L, M), dtype=np.complex128)
    if d == 2:
        ny, nx = x.shape
        Ex = np.exp(-1j * np.outer(k[:, 0], _r(nx)))   # [M, nx]
        Ey = np.exp(-1j * np.outer(k[:, 1], _r(ny)))   # [M, ny]
        for l in range(L):
            z = S[l] * x
            B = Ex @ z.T                                # [M, ny]
            y[l] = (B * Ey).sum(axis=1) * scale
        return y
    if d == 3:
        nz, ny, nx = x.shape
        for m0 in range(0, M, _CHUNK):
            kc = k[m0:m0 + _CHUNK]
            Ex = np.exp(-1j * np.outer(kc[:, 0], _r(nx)))
            Ey = np.exp(-1j * np.outer(kc[:, 1], _r(ny)))
            Ez = np.exp(-1j * np.outer(kc[:, 2], _r(nz)))
            for l in range(L):
                z = (S[l] * x).reshape(nz * ny, nx)
                B1 = (z @ Ex.T).reshape(nz, ny, -1)          # [nz, ny, mc]
                B2 = np.einsum("zym,my->zm", B1, Ey)          # [nz, mc]
                y[l, m0:m0 + _CHUNK] = np.einsum("zm,mz->m", B2, Ez) * scale
        return y
    raise ValueError("only 2D and 3D images are supported")


def adjoint(y, smaps, traj, dcf=None):
    """A^H D_w y: ``x[r] = N^{-1/2} sum_l conj(S_l[r]) sum_m w_m y_l[m] exp(+i<k_m, r>)``.

    y: ``[L][M]``; returns complex128 image shaped like ``smaps[0]``.
    """
    y = _as(y, np.complex128)
    S = _as(smaps, np.complex128)
    k = _as(traj, np.float64)
    shape = S.shape[1:]
    d = len(shape)
    N = int(np.prod(shape))
    L = S.shape[0]
    M = k.shape[0]
    w = np.ones(M) if dcf is None else _as(dcf, np.float64)
    scale = 1.0 / np.sqrt(N)
    out = np.zeros(shape, dtype=np.complex128)
    if d == 2:
        ny, nx = shape
        Exc = np.exp(1j * np.outer(k[:, 0], _r(nx)))    # [M, nx]
        Eyc = np.exp(1j * np.outer(k[:, 1], _r(ny)))    # [M, ny]
        for l in range(L):
            v = w * y[l]
            X = (Eyc * v[:, None]).T @ Exc              # [ny, nx]
            out += np.conj(S[l]) * X
        return out * scale
    if d == 3:
        nz, ny, nx = shape
        acc = np.zeros((L, nz, ny, nx), dtype=np.complex128)
        for m0 in range(0, M, _CHUNK):
            kc = k[m0:m0 + _CHUNK]
            Exc = np.exp(1j * np.outer(kc[:, 0], _r(nx)))
            Eyc = np.exp(1j * np.outer(kc[:, 1], _r(ny)))
            Ezc = np.exp(1j * np.outer(kc[:, 2], _r(nz)))
            for l in range(L):
                v = w[m0:m0 + _CHUNK] * y[l, m0:m0 + _CHUNK]
                Vzy = np.einsum("mz,my->mzy", Ezc * v[:, None], Eyc).reshape(-1, nz * ny)
                acc[l] += (Vzy.T @ Exc).reshape(nz, ny, nx)
        for l in range(L):
            out += np.conj(S[l]) * acc[l]
        return out * scale
    raise ValueError("only 2D and 3D images are supported")


def normal(x, smaps, traj, dcf=None):
    """A^H D_w A x (the normal operator of the weighted data term, Sec. 3.4)."""
    return adjoint(forward(x, smaps, traj), smaps, traj, dcf)


def forward_at(x, smaps, traj, sample_idx):
    """Exact A x restricted to the samples ``sample_idx`` (each output entry
    is independent of the others).  Returns ``[L][len(sample_idx)]``."""
    k = _as(traj, np.float64)[np.asarray(sample_idx)]
    return forward(x, smaps, k)


def adjoint_at(y, smaps, traj, dcf, flat_pixels):
    """Exact A^H D_w y at the flat pixel indices ``flat_pixels`` only.
    Returns complex128 ``[len(flat_pixels)]``."""
    y = _as(y, np.complex128)
    S = _as(smaps, np.complex128)
    k = _as(traj, np.float64)
    shape = S.shape[1:]
    N = int(np.prod(shape))
    M = k.shape[0]
    w = np.ones(M) if dcf is None else _as(dcf, np.float64)
    idx = np.unravel_index(np.asarray(flat_pixels), shape)     # slowest axis first
    # coordinates ordered (x, y[, z]) to match traj columns
    rc = np.stack([_r(shape[len(shape) - 1 - a])[idx[len(shape) - 1 - a]]
                   for a in range(len(shape))], axis=1)        # [P, d]
    out = np.zeros(len(rc), dtype=np.complex128)
    Sflat = S.reshape(S.shape[0], -1)[:, np.asarray(flat_pixels)]
    for p0 in range(0, len(rc), 256):
        E = np.exp(1j * (k @ rc[p0:p0 + 256].T))                 # [M, P]
        for l in range(S.shape[0]):
            out[p0:p0 + 256] += np.conj(Sflat[l, p0:p0 + 256]) * ((w * y[l]) @ E)
    return out / np.sqrt(N)


def dense_matrix(shape, smaps, traj):
    """Dense matrix of A (rows: (l, m) coil-major; columns: flat pixels),
    built entry by entry from the definition.  Tiny problems only."""
    S = _as(smaps, np.complex128)
    k = _as(traj, np.float64)
    L = S.shape[0]
    M = k.shape[0]
    N = int(np.prod(shape))
    coords = np.stack(np.meshgrid(*[_r(n) for n in shape], indexing="ij"), axis=-1).reshape(N, len(shape))
    coords = coords[:, ::-1]          # (x, y[, z]) order
    Amat = np.zeros((L * M, N), dtype=np.complex128)
    for l in range(L):
        for m in range(M):
            for p in range(N):
                Amat[l * M + m, p] = S[l].reshape(-1)[p] * np.exp(-1j * float(k[m] @ coords[p]))
    return Amat / np.sqrt(N)
