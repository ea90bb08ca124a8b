"""Power iteration, preconditioners, CG prox, annealed PnP-HQS and PnP-PGD.

All in FP64 on numpy arrays.  Every routine takes the operator as plain
callables, so the same code runs with the exact NDFT (``oracle.ndft``), a
dense matrix or any test operator:

* ``normal(v)`` -> A^H D_w A v
* ``b0``        =  A^H D_w y   (computed once by the caller)
* ``yw2``       =  ||y||^2_{D_w} = sum_l sum_m w_m |y_l[m]|^2 (for the residual)

Paper passages followed:
* data term f(x) = 1/2 sum_l ||F S_l x - y_l||^2 (Sec. 2.2), read with the
  DCF as a k-space weighting D_w; its gradient is A^H D_w (A x - y).
* PnP-HQS (Sec. 3.3):  u_k = prox^P_{gamma_k f}(x_k),  x_{k+1} = D_{sigma_k}(u_k)
* annealing (Sec. 3.3): sigma_k geometric, gamma_k = lambda * sigma_k
* metric prox (Sec. 3.4): prox^P_{gamma f}(x) = argmin_u gamma f(u) + 1/2 ||x-u||_P^2,
  computed by a sub-iteration solver: here conjugate gradients on the
  optimality condition (gamma A^H D_w A + P) u = P x + gamma b0, started at
  u = x, for a fixed number of steps.
* preconditioners (Sec. 3.4): F-1  P = 2 - alpha A^H A;  Chebyshev
  P = 4 - (10/3) A^H A (read with the same alpha normalisation);
  identity P = Id.  alpha = 1/||A^H D_w A||.
* PnP-PGD (Sec. 3.3):  u_k = x_k - gamma P grad f(x_k),  x_{k+1} = D_sigma(u_k)
* FISTA with the wavelet l1 prior (the FISTA-Wavelet baseline of Table 1):
  the accelerated proximal gradient method of Beck and Teboulle (2009) on
  f(x) + lam ||detail(Psi x)||_1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PRECOND = {"id": (1.0, 0.0), "f1": (2.0, 1.0), "cheb": (4.0, 10.0 / 3.0)}


def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(np.ravel(a), np.ravel(b)))


def precond_coeffs(name: str):
    """(c0, c1) with P = c0 I - c1 alpha A^H D_w A."""
    return PRECOND[name.lower()]


def precond_poly(name: str, t):
    """Scalar polynomial p(t) = c0 - c1 t of the preconditioner at a
    normalised eigenvalue t = alpha * lambda in [0, 1]."""
    c0, c1 = precond_coeffs(name)
    return c0 - c1 * np.asarray(t, dtype=np.float64)


def opnorm(normal, shape, seed: int = 0, tol: float = 1e-12, maxit: int = 1000):
    """||A^H D_w A||_2 by power iteration from a seeded complex Gaussian
    start, stopping when the Rayleigh quotient changes by less than ``tol``
    relative.  Returns (value, iterations)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    v /= np.linalg.norm(v)
    lam_old = 0.0
    for it in range(1, maxit + 1):
        w = normal(v)
        lam = vdot(v, w).real
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0, it
        v = w / nw
        if it > 1 and abs(lam - lam_old) <= tol * abs(lam):
            return lam, it
        lam_old = lam
    return lam, maxit


def opnorm_lanczos(normal, shape, tol: float = 1e-10, seed: int = 0):
    """||A^H D_w A||_2 as the largest eigenvalue of the Hermitian PSD normal
    operator by implicitly restarted Lanczos (ARPACK through scipy), which
    needs far fewer operator applications than power iteration when the top
    of the spectrum is clustered."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    n = int(np.prod(shape))
    op = LinearOperator((n, n), matvec=lambda v: np.ravel(normal(np.reshape(v, shape))),
                        dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    val = eigsh(op, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False)
    return float(val[0])


def cg_prox(x, b0, gamma: float, normal, c0: float, c1a: float, n_cg: int,
            Nx=None, trace=None):
    """prox^P_{gamma f}(x) by exactly ``n_cg`` CG steps (fewer only if the
    residual vanishes exactly).

    System: M u = b with M = gamma N + P = c0 I + (gamma - c1a) N,
    b = P x + gamma b0, N = A^H D_w A, c1a = c1 * alpha.  Start u0 = x, so
    r0 = b - M x = gamma (b0 - N x) (the P terms cancel).  ``Nx`` may pass
    N x when already known.  ``trace`` (a list) receives per-step
    (rr, pMp, a, beta) for diagnostics.
    """
    x = np.asarray(x, dtype=np.complex128)
    Nx = normal(x) if Nx is None else Nx

    def Mop(p):
        return c0 * p + (gamma - c1a) * normal(p)

    u = x.copy()
    r = gamma * (np.asarray(b0) - Nx)
    p = r.copy()
    rr = vdot(r, r).real
    for _ in range(n_cg):
        if rr == 0.0:
            break
        q = Mop(p)
        pq = vdot(p, q).real
        a = rr / pq
        u = u + a * p
        r = r - a * q
        rr_new = vdot(r, r).real
        beta = rr_new / rr
        if trace is not None:
            trace.append((rr, pq, a, beta))
        p = r + beta * p
        rr = rr_new
    return u


def dc_residual(x, Nx, b0, yw2: float) -> float:
    """rho = ||D_w^{1/2}(A x - y)||^2 = <x, N x> - 2 Re<x, b0> + ||y||^2_w."""
    return vdot(x, Nx).real - 2.0 * vdot(x, b0).real + yw2


@dataclass
class HQSReport:
    sigma: list = field(default_factory=list)
    gamma: list = field(default_factory=list)
    rho: list = field(default_factory=list)       # residual of x_k before step k+1
    fallback: list = field(default_factory=list)
    u_last: np.ndarray | None = None


def hqs(b0, normal, sigmas, lam: float, precond: str, n_cg: int, prior, opnorm_value: float,
        x0=None, yw2: float | None = None, fallback=None, rise_tol: float | None = None,
        report: HQSReport | None = None):
    """Annealed, preconditioned PnP-HQS (Sec. 3.3-3.4).

    ``prior(u, sigma)`` is the plug-in denoiser D_sigma.  For k = 1..n_out:
    gamma_k = lam * sigma_k; u_k = cg_prox(x_{k-1}); x_k = prior(u_k, sigma_k).

    Optional safeguard for learned priors: if ``fallback`` (a second prior)
    and ``rise_tol`` are given, then whenever x_k is non-finite or its
    data-consistency residual rho_k exceeds (1 + rise_tol) * rho_{k-1}, x_k
    is recomputed as fallback(u_k, sigma_k).  ``yw2`` (= ||y||^2_w) is needed
    for the residual.  Returns x_{n_out}.
    """
    c0, c1 = precond_coeffs(precond)
    c1a = c1 / opnorm_value
    x = np.array(b0 if x0 is None else x0, dtype=np.complex128, copy=True)
    Nx = normal(x)
    rho_prev = dc_residual(x, Nx, b0, yw2) if yw2 is not None else None
    for sigma in sigmas:
        gamma = lam * float(sigma)
        u = cg_prox(x, b0, gamma, normal, c0, c1a, n_cg, Nx=Nx)
        x = np.asarray(prior(u, float(sigma)), dtype=np.complex128)
        used_fb = False
        finite = bool(np.all(np.isfinite(x)))
        Nx = normal(x) if finite else None
        rho = dc_residual(x, Nx, b0, yw2) if (finite and yw2 is not None) else math.inf
        if fallback is not None and rise_tol is not None:
            if (not finite) or rho > (1.0 + rise_tol) * rho_prev:
                x = np.asarray(fallback(u, float(sigma)), dtype=np.complex128)
                Nx = normal(x)
                rho = dc_residual(x, Nx, b0, yw2)
                used_fb = True
        if report is not None:
            report.sigma.append(float(sigma))
            report.gamma.append(gamma)
            report.rho.append(rho)
            report.fallback.append(used_fb)
            report.u_last = u
        rho_prev = rho
    return x


def pgd(b0, normal, x0, gamma: float, n_iter: int, prior, sigma: float, precond: str = "id",
        opnorm_value: float = 1.0):
    """PnP-PGD (Sec. 3.3): u = x - gamma P grad f(x), x <- D_sigma(u), with
    grad f(x) = N x - b0 and P = c0 - c1 alpha N."""
    c0, c1 = precond_coeffs(precond)
    c1a = c1 / opnorm_value
    x = np.array(x0, dtype=np.complex128, copy=True)
    for _ in range(n_iter):
        g = normal(x) - b0
        Pg = c0 * g - c1a * normal(g) if c1 != 0.0 else c0 * g
        x = np.asarray(prior(x - gamma * Pg, sigma), dtype=np.complex128)
    return x


def pgd_schedule(b0, normal, x0, gamma: float, sigmas, prior, precond: str = "id", opnorm_value: float = 1.0):
    """PnP-PGD with one noise level per iteration (sigma_k of ``sigmas``),
    each step the PnP-PGD step of Sec. 3.3 at fixed gamma."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    for sigma in sigmas:
        x = pgd(b0, normal, x, gamma, 1, prior, float(sigma), precond, opnorm_value)
    return x


def fista(b0, normal, x0, gamma: float, n_iter: int, prox):
    """FISTA (Beck and Teboulle 2009) for f + g, f the data term with
    gradient N x - b0 and ``prox(v)`` = prox_{gamma g}(v):
        x_k     = prox(z_k - gamma (N z_k - b0))
        t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
        z_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1})
    from z_1 = x_0 and t_1 = 1.  Returns x_{n_iter}."""
    x_prev = np.array(x0, dtype=np.complex128, copy=True)
    z = x_prev.copy()
    t = 1.0
    for _ in range(n_iter):
        x = np.asarray(prox(z - gamma * (normal(z) - b0)), dtype=np.complex128)
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev, t = x, t_next
    return x_prev


def fista_wavelet(b0, normal, x0, gamma: float, lam: float, n_iter: int, levels: int | None = None):
    """FISTA on f(x) + lam ||detail(Psi x)||_1 (orthonormal Haar, detail bands
    only): the prox is the wavelet soft threshold at tau = gamma * lam."""
    from . import wavelet
    return fista(b0, normal, x0, gamma, n_iter, lambda v: wavelet.wavelet_denoise(v, gamma * lam, levels))
