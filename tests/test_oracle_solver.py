"""Pins of the oracle's Haar prior, CG prox, power iteration, preconditioners,
HQS/PGD loops and metrics against closed forms, dense linear algebra and the
fixed-point characterisation of Proposition 1 (Sec. 3.3)."""
import math

import numpy as np
import pytest

import synth
from oracle import ndft, solver, wavelet, metrics


# ----------------------------------------------------------------- Haar
def test_haar_one_level_known_values():
    x = np.array([[1.0, 3.0], [5.0, 7.0]])
    c = wavelet.haar_forward(x, 1)
    # 2x2 orthonormal Haar: approx = sum/2, then the three detail bands
    assert np.allclose(c, [[8.0, -2.0], [-4.0, 0.0]])
    v = np.array([[2.0, 4.0, 6.0, 8.0]] * 4)
    c = wavelet.haar_forward(v, 2)
    assert abs(c[0, 0] - v.sum() / 4) < 1e-14          # coarsest approx = sum / 2^J (2D)


@pytest.mark.parametrize("shape,J", [((64, 64), 3), ((48, 80), 4), ((16, 16, 32), 4)])
def test_haar_perfect_reconstruction_and_energy(shape, J):
    x = synth.white_complex(shape, 30).astype(np.complex128)
    c = wavelet.haar_forward(x, J)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.max(np.abs(wavelet.haar_inverse(c, J) - x)) < 1e-13


def test_haar_matches_block_averages():
    # approximation band after J levels = block sums / 2^J for 2^J x 2^J blocks
    x = synth.white_complex((32, 32), 31).astype(np.complex128)
    J = 3
    c = wavelet.haar_forward(x, J)
    blocks = x.reshape(4, 8, 4, 8).sum(axis=(1, 3)) / 2 ** J
    assert np.allclose(c[:4, :4], blocks, atol=1e-13)


def test_soft_threshold_is_l1_prox():
    rng = np.random.default_rng(0)
    tau = 0.3
    for _ in range(20):
        c = complex(*rng.normal(size=2))
        s = wavelet.soft_threshold(np.array([c]), tau)[0]
        # brute-force argmin_v tau|v| + 1/2|c - v|^2 over a fine grid around c
        g = np.linspace(-3, 3, 1201)
        V = g[:, None] + 1j * g[None, :]
        obj = tau * np.abs(V) + 0.5 * np.abs(c - V) ** 2
        vb = V.ravel()[np.argmin(obj)]
        assert abs(s - vb) < 6e-3
        # subgradient optimality: c - s in tau * d|s|
        if s != 0:
            assert abs((c - s) - tau * s / abs(s)) < 1e-12
        else:
            assert abs(c) <= tau


def test_wavelet_prior_special_cases():
    x = synth.white_complex((32, 32), 32).astype(np.complex128)
    assert np.max(np.abs(wavelet.wavelet_denoise(x, 0.0, 2) - x)) < 1e-13
    # huge threshold: only the approximation band survives = block means
    y = wavelet.wavelet_denoise(x, 1e9, 2)
    means = x.reshape(8, 4, 8, 4).mean(axis=(1, 3))
    assert np.allclose(y, np.kron(means, np.ones((4, 4))), atol=1e-13)


def test_wavelet_prior_is_prox_of_detail_l1():
    # D(u) minimises tau*||detail(Hv)||_1 + 1/2||u - v||^2: random perturbations never do better
    u = synth.white_complex((16, 16), 33).astype(np.complex128)
    tau, J = 0.4, 2
    v = wavelet.wavelet_denoise(u, tau, J)
    f = lambda z: tau * wavelet.l1_detail(z, J) + 0.5 * np.linalg.norm(u - z) ** 2
    f0 = f(v)
    rng = np.random.default_rng(1)
    for _ in range(50):
        d = (rng.normal(size=u.shape) + 1j * rng.normal(size=u.shape)) * 1e-3
        assert f(v + d) >= f0 - 1e-12


def test_default_levels():
    assert wavelet.default_levels(64) == 3
    assert wavelet.default_levels(320) == 4
    assert wavelet.default_levels(128) == 4


# ------------------------------------------------------------ operators
def _tiny_problem(n=8, L=2, M=40, seed=40):
    rng = np.random.default_rng(seed)
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    S = synth.smaps2d(n, L)
    w = rng.uniform(0.5, 1.5, M)
    A = ndft.dense_matrix((n, n), S, k)
    Wd = np.kron(np.eye(L), np.diag(w))
    Nmat = A.conj().T @ Wd @ A
    normal = lambda v: ndft.normal(v, S, k, w)
    return k, S, w, A, Nmat, normal


def test_power_iteration_equals_max_eigenvalue():
    k, S, w, A, Nmat, normal = _tiny_problem()
    lam, its = solver.opnorm(normal, (8, 8), seed=3, tol=1e-13, maxit=5000)
    ev = np.linalg.eigvalsh(Nmat)
    assert abs(lam - ev[-1]) < 1e-9 * ev[-1]
    assert ev[0] > -1e-12          # PSD


def test_normal_operator_hermitian_psd():
    k, S, w, A, Nmat, normal = _tiny_problem()
    x = synth.white_complex((8, 8), 41)
    q = np.vdot(x.astype(np.complex128), normal(x))
    assert q.real > 0 and abs(q.imag) < 1e-12 * q.real
    assert np.allclose(Nmat, Nmat.conj().T, atol=1e-13)


@pytest.mark.parametrize("name,c0,c1,tmax_p", [("f1", 2.0, 1.0, 1.0), ("cheb", 4.0, 10 / 3, 1.2)])
def test_preconditioner_polynomials(name, c0, c1, tmax_p):
    assert solver.precond_coeffs(name) == (c0, c1)
    t = np.linspace(1e-6, 1, 10001)
    p = solver.precond_poly(name, t)
    tp = t * p
    assert tp.min() > 0 and tp.max() <= tmax_p + 1e-12
    assert p.min() >= (1.0 if name == "f1" else 2.0 / 3.0) - 1e-12     # P is positive definite
    # design rule: the spectral radius of Id - alpha P A^H A over a spectrum
    # [t0, 1] is smaller than with P = Id
    for t0 in (0.01, 0.05, 0.2):
        sel = t >= t0
        assert np.abs(1 - tp[sel]).max() < np.abs(1 - t[sel]).max()
    if name == "f1":
        assert np.allclose(1 - tp, (1 - t) ** 2)


@pytest.mark.parametrize("precond", ["id", "f1", "cheb"])
def test_cg_prox_converges_to_dense_solve(precond):
    k, S, w, A, Nmat, normal = _tiny_problem()
    Lnorm = np.linalg.eigvalsh(Nmat)[-1]
    c0, c1 = solver.precond_coeffs(precond)
    P = c0 * np.eye(64) - c1 / Lnorm * Nmat
    x = synth.white_complex((8, 8), 42).astype(np.complex128)
    y = synth.white_complex((2, 40), 43).astype(np.complex128)
    b0 = ndft.adjoint(y, S, k, w)
    gamma = 0.7
    u = solver.cg_prox(x, b0, gamma, normal, c0, c1 / Lnorm, n_cg=200)
    # u = argmin gamma f_w(u) + 1/2 ||x - u||_P^2  <=>  (gamma N + P) u = P x + gamma b0
    u_ref = np.linalg.solve(gamma * Nmat + P, P @ x.ravel() + gamma * b0.ravel())
    assert np.max(np.abs(u.ravel() - u_ref)) < 1e-10
    # stationarity of the prox objective
    g = gamma * (A.conj().T @ (np.kron(np.eye(2), np.diag(w)) @ (A @ u.ravel() - y.ravel()))) + P @ (u.ravel() - x.ravel())
    assert np.linalg.norm(g) < 1e-9


@pytest.mark.parametrize("precond,c0p", [("id", 1.0), ("f1", 1.0), ("cheb", 2.0 / 3.0)])
def test_cg_prox_closed_form_identity_normal(precond, c0p):
    """Full Cartesian sampling with SoS-1 maps gives A^H A = I, ||N|| = 1, so
    P = c0' I and the prox has the closed form (c0' x + gamma b0)/(gamma + c0'),
    reached by one CG step."""
    n = 8
    S = synth.smaps2d(n, 3).astype(np.complex128)
    S /= np.sqrt((np.abs(S) ** 2).sum(0))
    k = synth.cartesian2d(n, np.float64)
    normal = lambda v: ndft.normal(v, S, k)
    x = synth.white_complex((n, n), 44).astype(np.complex128)
    b0 = synth.white_complex((n, n), 45).astype(np.complex128)
    c0, c1 = solver.precond_coeffs(precond)
    gamma = 0.37
    u = solver.cg_prox(x, b0, gamma, normal, c0, c1 * 1.0, n_cg=1)
    assert np.max(np.abs(u - (c0p * x + gamma * b0) / (gamma + c0p))) < 1e-12


def test_dc_residual_two_forms():
    k, S, w, A, Nmat, normal = _tiny_problem()
    x = synth.white_complex((8, 8), 46).astype(np.complex128)
    y = synth.white_complex((2, 40), 47).astype(np.complex128)
    b0 = ndft.adjoint(y, S, k, w)
    yw2 = float((w[None] * np.abs(y) ** 2).sum())
    r_direct = float((w[None] * np.abs(ndft.forward(x, S, k) - y) ** 2).sum())
    r_fast = solver.dc_residual(x, normal(x), b0, yw2)
    assert abs(r_direct - r_fast) < 1e-12 * r_direct


def test_hqs_identity_prior_is_proximal_point_to_least_squares():
    """P = Id and D = identity: HQS is the proximal-point method on f, whose
    iterates approach a least-squares solution (textbook)."""
    k, S, w, A, Nmat, normal = _tiny_problem(M=120)
    y = synth.white_complex((2, 120), 48).astype(np.complex128)
    b0 = ndft.adjoint(y, S, k, w)
    x = solver.hqs(b0, normal, [1.0] * 60, lam=5.0, precond="id", n_cg=300,
                   prior=lambda u, s: u, opnorm_value=np.linalg.eigvalsh(Nmat)[-1])
    x_ls = np.linalg.lstsq(Nmat, b0.ravel(), rcond=None)[0]
    assert np.linalg.norm(Nmat @ x.ravel() - b0.ravel()) < 1e-8 * np.linalg.norm(b0)
    assert np.linalg.norm(x.ravel() - x_ls) < 1e-6 * np.linalg.norm(x_ls)


def test_proposition1_fixed_points():
    """Proposition 1 with D = prox_g (g = tau * l1 of Haar details, convex),
    P = Id, constant gamma and sigma:
    * HQS's u-iterate converges to argmin gamma f + (Moreau envelope of g),
      i.e. gamma grad f(u*) + u* - prox_g(u*) = 0;
    * PnP-PGD converges to argmin gamma f + g, i.e. x* = prox_g(x* - gamma grad f(x*))."""
    n = 8
    rng = np.random.default_rng(49)
    M = 200          # 400 equations for 64 unknowns: f is strongly convex
    k = rng.uniform(-math.pi, math.pi, (M, 2))
    S = synth.smaps2d(n, 2)
    normal = lambda v: ndft.normal(v, S, k)
    xt, _ = synth.phantom2d(n, 5)
    y = ndft.forward(xt, S, k) + synth.complex_noise((2, M), 1e-4, 6)
    b0 = ndft.adjoint(y, S, k)
    Ln, _ = solver.opnorm(normal, (n, n), tol=1e-12)
    tau = 0.02
    prox_g = lambda v, s: wavelet.wavelet_denoise(v, tau, 2)
    gamma = 1.0 / Ln
    rep = solver.HQSReport()
    solver.hqs(b0, normal, [1.0] * 200, lam=gamma, precond="id", n_cg=70, prior=prox_g,
               opnorm_value=Ln, report=rep)
    u = rep.u_last
    res = gamma * (normal(u) - b0) + u - prox_g(u, 1.0)
    assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(u)
    # PGD fixed point (step gamma < 2/L)
    x = solver.pgd(b0, normal, b0, gamma, 300, prox_g, 1.0)
    fp = prox_g(x - gamma * (normal(x) - b0), 1.0)
    assert np.linalg.norm(fp - x) < 1e-10 * np.linalg.norm(x)
    # and the two limits differ (the paper's point)
    assert np.linalg.norm(prox_g(u, 1.0) - x) > 1e-6 * np.linalg.norm(x)


def test_fista_scalar_hand_iterates():
    """Three FISTA steps on the scalar problem a/2 x^2 - b x + tau |x| (a = 0.5,
    b = 2, tau = 0.1, gamma = 1, x0 = 0), iterates worked by hand:
    x1 = soft(2) = 1.9, z2 = 1.9 (t1 = 1); x2 = soft(2.95) = 2.85,
    t2 = (1 + sqrt 5)/2, z3 = 2.85 + (t2 - 1)/t3 * 0.95 = 3.117665849;
    x3 = soft(3.558832924) = 3.458832924.  The limit is (b - tau)/a = 3.8."""
    a, b, tau = 0.5, 2.0, 0.1
    normal = lambda v: a * v
    b0 = np.array([b], dtype=np.complex128)
    soft = lambda v: np.sign(v) * np.maximum(np.abs(v) - tau, 0.0)
    got = [solver.fista(b0, normal, np.zeros(1), 1.0, k, soft)[0].real for k in (1, 2, 3)]
    assert np.allclose(got, [1.9, 2.85, 3.4588329244345273], rtol=0, atol=1e-12)
    assert abs(solver.fista(b0, normal, np.zeros(1), 1.0, 400, soft)[0] - 3.8) < 1e-9


def test_fista_wavelet_identity_normal_closed_form():
    """A^H D_w A = Id: the minimiser of 1/2 ||x - b0||^2 + lam ||detail(Psi x)||_1 is
    the wavelet soft threshold of b0 at lam (orthonormal Psi); FISTA with
    gamma = 1 reaches it in one step, with gamma = 0.4 in the limit."""
    b0 = synth.white_complex((16, 16), 61).astype(np.complex128)
    lam = 0.3
    ref = wavelet.wavelet_denoise(b0, lam, 2)
    one = solver.fista_wavelet(b0, lambda v: v, np.zeros_like(b0), 1.0, lam, 1, 2)
    assert np.abs(one - ref).max() < 1e-14
    lim = solver.fista_wavelet(b0, lambda v: v, np.zeros_like(b0), 0.4, lam, 300, 2)
    assert np.abs(lim - ref).max() < 1e-10


def test_fista_wavelet_reaches_the_pgd_minimiser():
    """On a strongly convex NUFFT problem, FISTA-Wavelet and plain proximal
    gradient (the PGD loop with D = prox) converge to the same minimiser of
    f + lam ||detail(Psi x)||_1 (unique), which satisfies the fixed-point
    condition x = prox(x - gamma grad f(x))."""
    n = 8
    rng = np.random.default_rng(62)
    M = 200
    k = rng.uniform(-math.pi, math.pi, (M, 2))
    S = synth.smaps2d(n, 2)
    normal = lambda v: ndft.normal(v, S, k)
    xt, _ = synth.phantom2d(n, 7)
    y = ndft.forward(xt, S, k) + synth.complex_noise((2, M), 1e-4, 8)
    b0 = ndft.adjoint(y, S, k)
    Ln, _ = solver.opnorm(normal, (n, n), tol=1e-12)
    gamma, lam = 1.0 / Ln, 0.05
    xf = solver.fista_wavelet(b0, normal, b0, gamma, lam, 400, 2)
    prox = lambda v, s: wavelet.wavelet_denoise(v, gamma * lam, 2)
    xp = solver.pgd(b0, normal, b0, gamma, 3000, prox, 1.0)
    assert np.linalg.norm(xf - xp) < 1e-9 * np.linalg.norm(xp)
    fp = prox(xf - gamma * (normal(xf) - b0), 1.0)
    assert np.linalg.norm(fp - xf) < 1e-9 * np.linalg.norm(xf)
    # acceleration: after 30 steps FISTA is closer to the minimiser than proximal gradient
    e_f = np.linalg.norm(solver.fista_wavelet(b0, normal, b0, gamma, lam, 30, 2) - xp)
    e_p = np.linalg.norm(solver.pgd(b0, normal, b0, gamma, 30, prox, 1.0) - xp)
    assert e_f < e_p


def test_lanczos_norm_equals_max_eigenvalue():
    """The Lanczos (ARPACK) norm is the top eigenvalue of the dense normal
    matrix, and agrees with the power-iteration norm; a wrong eigenvalue
    choice (smallest, or the largest in magnitude of a shifted matrix) or a
    dropped DCF weighting would not."""
    k, S, w, A, Nmat, normal = _tiny_problem()
    ev = np.linalg.eigvalsh(Nmat)
    lam = solver.opnorm_lanczos(normal, (8, 8), tol=1e-12, seed=5)
    assert abs(lam - ev[-1]) < 1e-10 * ev[-1]
    lam_p, _ = solver.opnorm(normal, (8, 8), seed=3, tol=1e-13, maxit=5000)
    assert abs(lam - lam_p) < 1e-9 * ev[-1]
    # the weighting matters: the unweighted operator has another norm
    ev_u = np.linalg.eigvalsh(A.conj().T @ A)[-1]
    assert abs(ev_u - ev[-1]) > 1e-3 * ev[-1]
    # full Cartesian sampling with SoS-1 maps: A^H A = I, so the norm is 1
    n = 8
    Sc = synth.smaps2d(n, 3).astype(np.complex128)
    Sc /= np.sqrt((np.abs(Sc) ** 2).sum(0))
    kc = synth.cartesian2d(n, np.float64)
    assert abs(solver.opnorm_lanczos(lambda v: ndft.normal(v, Sc, kc), (n, n)) - 1.0) < 1e-10


@pytest.mark.parametrize("precond", ["f1", "cheb"])
def test_preconditioned_pgd_step_dense(precond):
    """One PnP-PGD step with the identity denoiser against the dense formula
    x - gamma (c0 I - c1 alpha N)(N x - b0), N the dense normal matrix built
    from the brute-force NDFT matrix (Sec. 3.3 PnP-PGD with the Sec. 3.4
    preconditioners).  A flipped sign of the c1 term, a dropped alpha or a
    preconditioner applied to x instead of the gradient each fail."""
    k, S, w, A, Nmat, normal = _tiny_problem()
    Ln = np.linalg.eigvalsh(Nmat)[-1]
    c0, c1 = {"f1": (2.0, 1.0), "cheb": (4.0, 10.0 / 3.0)}[precond]
    P = c0 * np.eye(64) - (c1 / Ln) * Nmat
    x = synth.white_complex((8, 8), 64).astype(np.complex128)
    b0 = synth.white_complex((8, 8), 65).astype(np.complex128)
    gamma = 0.8 / Ln
    got = solver.pgd(b0, normal, x, gamma, 1, lambda u, s: u, 0.0, precond, Ln)
    ref = x.ravel() - gamma * (P @ (Nmat @ x.ravel() - b0.ravel()))
    assert np.max(np.abs(got.ravel() - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("precond", ["f1", "cheb"])
def test_preconditioned_pgd_reaches_least_squares(precond):
    """With D = identity, preconditioned gradient descent x <- x - gamma P (N x - b0)
    converges to the least-squares solution N x = b0 (strongly convex tiny
    problem), and faster than P = Id at the same gamma (the point of the
    preconditioner, Sec. 3.4)."""
    k, S, w, A, Nmat, normal = _tiny_problem(M=120)
    y = synth.white_complex((2, 120), 66).astype(np.complex128)
    b0 = ndft.adjoint(y, S, k, w)
    Ln = np.linalg.eigvalsh(Nmat)[-1]
    x_ls = np.linalg.solve(Nmat, b0.ravel())
    ident = lambda u, s: u
    gamma = 1.0 / Ln
    # F-1: t p(t) <= 1 on [0, 1], Chebyshev: <= 1.2, so gamma = 1/L is a stable step for both
    x = solver.pgd(b0, normal, b0, gamma, 4000, ident, 0.0, precond, Ln)
    assert np.linalg.norm(x.ravel() - x_ls) < 1e-8 * np.linalg.norm(x_ls)
    e_pre = np.linalg.norm(solver.pgd(b0, normal, b0, gamma, 40, ident, 0.0, precond, Ln).ravel() - x_ls)
    e_id = np.linalg.norm(solver.pgd(b0, normal, b0, gamma, 40, ident, 0.0, "id", Ln).ravel() - x_ls)
    assert e_pre < e_id


def test_pgd_schedule_constant_equals_pgd():
    k, S, w, A, Nmat, normal = _tiny_problem()
    b0 = synth.white_complex((8, 8), 63).astype(np.complex128)
    prior = lambda u, s: wavelet.wavelet_denoise(u, 0.1 * s, 2)
    Ln = np.linalg.eigvalsh(Nmat)[-1]
    a = solver.pgd(b0, normal, b0, 0.5 / Ln, 7, prior, 0.3, "f1", Ln)
    b = solver.pgd_schedule(b0, normal, b0, 0.5 / Ln, [0.3] * 7, prior, "f1", Ln)
    assert np.abs(a - b).max() < 1e-15


def test_hqs_fallback_on_bad_prior():
    """A prior that returns garbage raises the residual; the fallback
    (wavelet) takes over and the final result equals the all-wavelet run."""
    k, S, w, A, Nmat, normal = _tiny_problem(M=100)
    y = synth.white_complex((2, 100), 50).astype(np.complex128)
    b0 = ndft.adjoint(y, S, k, w)
    yw2 = float((w[None] * np.abs(y) ** 2).sum())
    Ln = np.linalg.eigvalsh(Nmat)[-1]
    wav = lambda u, s: wavelet.wavelet_denoise(u, 0.1 * s, 1)
    bad = lambda u, s: u * 0 + np.nan
    sig = synth.geometric_sigmas(0.1, 0.01, 6)
    rep = solver.HQSReport()
    xa = solver.hqs(b0, normal, sig, 3.0, "f1", 3, bad, Ln, yw2=yw2, fallback=wav, rise_tol=0.5, report=rep)
    xb = solver.hqs(b0, normal, sig, 3.0, "f1", 3, wav, Ln, yw2=yw2)
    assert all(rep.fallback)
    assert np.max(np.abs(xa - xb)) < 1e-13


def test_geometric_schedule():
    s = synth.geometric_sigmas(0.1, 0.005, 30)
    assert abs(s[0] - 0.1) < 1e-15 and abs(s[-1] - 0.005) < 1e-15
    assert abs(s[1] / s[0] - 0.90186) < 1e-5


# -------------------------------------------------------------- metrics
def test_psnr_constant_offset():
    x = np.ones((16, 16)) * 0.8
    xh = x + 0.01
    roi = np.ones_like(x, dtype=bool)
    assert abs(metrics.psnr(xh, x, roi) - 20 * math.log10(0.8 / 0.01)) < 1e-9
    roi[:8] = False
    assert abs(metrics.psnr(xh, x, roi) - 20 * math.log10(0.8 / 0.01)) < 1e-9


def test_ssim_identical_and_constant():
    x, _ = synth.phantom2d(32, 3)
    assert abs(metrics.ssim(x, x) - 1) < 1e-12
    a = np.full((20, 20), 0.5)
    b = np.full((20, 20), 1.0)
    # constant images: variances 0 -> SSIM = luminance term (2ab + C1)/(a^2 + b^2 + C1)
    C1 = (0.01 * 1.0) ** 2
    exp = (2 * 0.5 * 1.0 + C1) / (0.25 + 1.0 + C1)
    assert abs(metrics.ssim(a, b) - exp) < 1e-12
