"""GPU parity of PnP-PGD (Sec. 3.3) and FISTA-Wavelet (the wavelet baseline
of Table 1) against the FP64 oracle (exact NDFT operator).  Bar for the
final image: relative L2 <= 1e-4, as for HQS (FP32 arithmetic over a few
tens of operator applications)."""
import numpy as np
import pytest

import synth
from oracle import ndft, solver, wavelet
from tests.golden import make_golden
from tests.gpu_util import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


def _problem(w, seed):
    x, roi = synth.phantom2d(w.n, seed)
    S = synth.smaps2d(w.n, w.L)
    k = w.traj.k
    dcf = synth.voronoi_dcf(w.traj, w.n) if w.dcf else None
    nu = synth.noise_variance(x, S)
    y = ndft.forward(x, S, k) + synth.complex_noise((w.L, k.shape[0]), nu, synth.SEED_NOISE + seed)
    return x, roi, S, k, dcf, y.astype(np.complex64)


def _opnorm(w, normal):
    if w.n == 320:
        return make_golden.load_opnorm()
    return solver.opnorm(normal, (w.n, w.n), tol=1e-12, maxit=3000)[0]


@pytest.mark.parametrize("precond,toeplitz", [("id", False), ("f1", False), ("cheb", True), ("f1", True)])
def test_pgd_tiny_matches_oracle(pnp, precond, toeplitz):
    w = synth.config_tiny()
    x, roi, S, k, dcf, y = _problem(w, 11)
    normal = lambda v: ndft.normal(v, S, k, dcf)
    Ln = _opnorm(w, normal)
    b0 = ndft.adjoint(y, S, k, dcf)
    kappa = 0.5
    sig = synth.geometric_sigmas(0.05, 0.005, 8)
    # step within the stable range of each preconditioned gradient map
    gamma = {"id": 1.0, "f1": 1.0, "cheb": 0.8}[precond] / Ln
    prior_o = lambda u, s: wavelet.wavelet_denoise(u, kappa * s)
    x_ref = solver.pgd_schedule(b0, normal, b0, gamma, sig, prior_o, precond, Ln)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    dd = to_dev(dcf) if dcf is not None else None
    tp = pnp.Toeplitz(plan, dd) if toeplitz else None
    xg = to_np(pnp.pgd_solve(plan, to_dev(y), to_dev(S), dd, pnp.WaveletPrior(0, kappa), sig, gamma, precond,
                             opnorm=Ln, toeplitz=tp))
    e = rel_l2(xg, x_ref)
    say(f"[pgd] tiny P={precond} toeplitz={toeplitz} {len(sig)} its: image rel {e:.3e}")
    assert e < TOL


def test_pgd_clinical_matches_oracle(pnp):
    """320x320, 16 coils, spiral + Voronoi DCF, F-1, Toeplitz; 3 iterations
    (6 normal operators in the oracle)."""
    w = synth.config_clinical()
    x, roi, S, k, dcf, y = _problem(w, 12)
    normal = lambda v: ndft.normal(v, S, k, dcf)
    Ln = _opnorm(w, normal)
    b0 = ndft.adjoint(y, S, k, dcf)
    sig = [0.02, 0.015, 0.01]
    gamma = 1.0 / Ln
    prior_o = lambda u, s: wavelet.wavelet_denoise(u, 0.75 * s)
    x_ref = solver.pgd_schedule(b0, normal, b0, gamma, sig, prior_o, "f1", Ln)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    dd = to_dev(dcf)
    xg = to_np(pnp.pgd_solve(plan, to_dev(y), to_dev(S), dd, pnp.WaveletPrior(0, 0.75), sig, gamma, "f1",
                             opnorm=Ln, toeplitz=pnp.Toeplitz(plan, dd)))
    e = rel_l2(xg, x_ref)
    say(f"[pgd] clinical F-1 Toeplitz 3 its: image rel {e:.3e}")
    assert e < TOL


@pytest.mark.parametrize("toeplitz", [False, True])
def test_fista_wavelet_tiny_matches_oracle(pnp, toeplitz):
    w = synth.config_tiny()
    x, roi, S, k, dcf, y = _problem(w, 13)
    normal = lambda v: ndft.normal(v, S, k, dcf)
    Ln = _opnorm(w, normal)
    b0 = ndft.adjoint(y, S, k, dcf)
    gamma = 1.0 / Ln
    lam = 0.02 * float(np.abs(b0).max()) * Ln
    x_ref = solver.fista_wavelet(b0, normal, b0, gamma, lam, 12)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    dd = to_dev(dcf) if dcf is not None else None
    tp = pnp.Toeplitz(plan, dd) if toeplitz else None
    xg = to_np(pnp.fista_wavelet(plan, to_dev(y), to_dev(S), dd, lam, gamma, 12, toeplitz=tp))
    e = rel_l2(xg, x_ref)
    say(f"[fista] tiny toeplitz={toeplitz} 12 its: image rel {e:.3e}")
    assert e < TOL


def test_fista_wavelet_clinical_matches_oracle(pnp):
    w = synth.config_clinical()
    x, roi, S, k, dcf, y = _problem(w, 14)
    normal = lambda v: ndft.normal(v, S, k, dcf)
    Ln = _opnorm(w, normal)
    b0 = ndft.adjoint(y, S, k, dcf)
    gamma = 1.0 / Ln
    lam = 0.01 * float(np.abs(b0).max()) * Ln
    x_ref = solver.fista_wavelet(b0, normal, b0, gamma, lam, 4)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    dd = to_dev(dcf)
    xg = to_np(pnp.fista_wavelet(plan, to_dev(y), to_dev(S), dd, lam, gamma, 4, toeplitz=pnp.Toeplitz(plan, dd)))
    e = rel_l2(xg, x_ref)
    say(f"[fista] clinical Toeplitz 4 its: image rel {e:.3e}")
    assert e < TOL


def test_pgd_rejects_bad_arguments(pnp):
    w = synth.config_tiny()
    x, roi, S, k, dcf, y = _problem(w, 15)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    with pytest.raises(pnp.PnPError):
        pnp.pgd_solve(plan, to_dev(y), to_dev(S), None, pnp.WaveletPrior(0, 0.5), [0.1], 0.5, "f1", opnorm=0.0)
    with pytest.raises(pnp.PnPError):
        pnp.fista_wavelet(plan, to_dev(y), to_dev(S), None, -1.0, 0.5, 3)
