"""3D operators and HQS against the FP64 oracle.

Small volumes (64^3 and a non-cubic 64 x 64 x 128) are compared element by
element with the exact NDFT (bar 2e-5 per operator; 1e-4 for the HQS
image).  At the full 128^3 / 32-coil / 4,096 x 256 kooshball size the
oracle computes sampled outputs one by one (forward at random samples,
adjoint at random voxels), and the Toeplitz normal operator is checked
against the gridded one and for self-adjointness."""
import numpy as np
import pytest

import synth
from oracle import ndft, solver, wavelet
from tests.gpu_util import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu
TOL = 2e-5


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


def _kball(spokes, S, seed=None):
    k = synth.kooshball3d(spokes, S).k
    return k


@pytest.mark.parametrize("shape,L,spokes,S", [((64, 64, 64), 2, 64, 128), ((64, 64, 128), 3, 40, 96)])
def test_3d_operators_match_ndft(pnp, shape, L, spokes, S):
    k = _kball(spokes, S)
    M = k.shape[0]
    x = synth.white_complex(shape, 1)
    Smaps = synth.white_complex((L,) + shape, 2)
    dcf = np.random.default_rng(3).uniform(0.5, 1.5, M).astype(np.float32)
    plan = pnp.Plan(to_dev(k), shape)
    xd, Sd, dd = to_dev(x), to_dev(Smaps), to_dev(dcf)
    e_f = rel_l2(to_np(plan.forward(xd, Sd)), ndft.forward(x, Smaps, k))
    y = synth.white_complex((L, M), 4)
    e_a = rel_l2(to_np(plan.adjoint(to_dev(y), Sd, dd)), ndft.adjoint(y, Smaps, k, dcf))
    ref_n = ndft.normal(x, Smaps, k, dcf)
    e_n = rel_l2(to_np(plan.normal(xd, Sd, dd)), ref_n)
    e_t = rel_l2(to_np(pnp.Toeplitz(plan, dd).normal(xd, Sd)), ref_n)
    say(f"[3d] {shape} L={L} M={M}: forward {e_f:.2e} adjoint {e_a:.2e} normal {e_n:.2e} toeplitz {e_t:.2e}")
    assert max(e_f, e_a, e_n, e_t) < TOL


def test_3d_hqs_matches_oracle(pnp):
    n, L = 64, 2
    k = _kball(64, 128)
    M = k.shape[0]
    x, roi = synth.phantom3d(n, 5)
    Smaps = synth.smaps3d(n, L)
    y = (ndft.forward(x, Smaps, k) + synth.complex_noise((L, M), synth.noise_variance(x, Smaps), 6)).astype(
        np.complex64)
    normal = lambda v: ndft.normal(v, Smaps, k)
    Ln, _ = solver.opnorm(normal, (n, n, n), tol=1e-10, maxit=300)
    sig = synth.geometric_sigmas(0.1, 0.005, 20)[:2]
    lam = 300.0 / Ln
    b0 = ndft.adjoint(y, Smaps, k)

    def prior_o(u, s):
        say(f"   oracle 3D outer step sigma={s:.4f}")
        return wavelet.wavelet_denoise(u, 0.75 * s)
    x_ref = solver.hqs(b0, normal, sig, lam, "f1", 3, prior_o, Ln)
    plan = pnp.Plan(to_dev(k), (n, n, n))
    tp = pnp.Toeplitz(plan)
    xg, _ = pnp.hqs_solve(plan, to_dev(y), to_dev(Smaps), None, pnp.WaveletPrior(0, 0.75), sig, lam, "f1", 3,
                          opnorm=Ln, toeplitz=tp)
    e = rel_l2(to_np(xg), x_ref)
    say(f"[3d] HQS 64^3 L=2, 2 outer x 3 CG (Toeplitz): image rel {e:.2e}")
    assert e < 1e-4


@pytest.mark.slow
def test_3d_full_size_sampled(pnp):
    """128^3, 32 coils, 4,096 x 256 kooshball: sampled parity and properties."""
    w = synth.config_3d()
    n, L = w.n, w.L
    k = w.traj.k
    M = k.shape[0]
    x, _ = synth.phantom3d(n, 7)
    Smaps = synth.smaps3d(n, L)
    plan = pnp.Plan(to_dev(k), (n, n, n))
    xd, Sd = to_dev(x), to_dev(Smaps)
    y = to_np(plan.forward(xd, Sd))
    rng = np.random.default_rng(8)
    idx = rng.choice(M, 12, replace=False)
    ref = ndft.forward_at(x, Smaps, k, idx)
    e_f = rel_l2(y[:, idx], ref)
    yv = synth.white_complex((L, M), 9)
    dcf = synth.radial3d_dcf(w.traj, n)
    xa = to_np(plan.adjoint(to_dev(yv), Sd, to_dev(dcf)))
    vox = rng.choice(n ** 3, 6, replace=False)
    ref_a = ndft.adjoint_at(yv, Smaps, k, dcf, vox)
    e_a = rel_l2(xa.reshape(-1)[vox], ref_a)
    tp = pnp.Toeplitz(plan, to_dev(dcf))
    Nt = to_np(tp.normal(xd, Sd)).astype(np.complex128)
    Ng = to_np(plan.normal(xd, Sd, to_dev(dcf))).astype(np.complex128)
    e_tg = rel_l2(Nt, Ng)
    x2 = synth.white_complex((n, n, n), 10)
    Nt2 = to_np(tp.normal(to_dev(x2), Sd)).astype(np.complex128)
    lhs, rhs = np.vdot(x2.astype(np.complex128), Nt), np.vdot(Nt2, x.astype(np.complex128))
    e_sa = abs(lhs - rhs) / abs(lhs)
    say(f"[3d] 128^3 L=32 M={M}: forward@12 samples {e_f:.2e}, adjoint@6 voxels {e_a:.2e}, "
        f"Toeplitz vs gridded {e_tg:.2e}, self-adjoint {e_sa:.2e}")
    assert max(e_f, e_a, e_tg) < TOL
    assert e_sa < 1e-5
