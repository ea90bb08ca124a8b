"""GPU parity of A, A^H D_w and A^H D_w A against the exact FP64 NDFT oracle.

Bar: relative L2 error <= 2e-5 per operator application (FP32 Kaiser-Bessel
gridding, W = 6, oversampling 2, against the exact transform)."""
import math

import numpy as np
import pytest

import synth
from oracle import ndft
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


def _case(n, L, traj, seed, dcf=None):
    x, _ = synth.phantom2d(n, seed)
    S = synth.smaps2d(n, L)
    return x, S, traj, dcf


def _run_ops(pnp, shape, x, S, k, dcf, label):
    say(f"[ops] {label}: shape={shape} L={S.shape[0]} M={k.shape[0]}")
    plan = pnp.Plan(to_dev(k), shape)
    xd, Sd = to_dev(x), to_dev(S)
    dd = to_dev(dcf) if dcf is not None else None
    y = to_np(plan.forward(xd, Sd))
    y_ref = ndft.forward(x, S, k)
    e_f = rel_l2(y, y_ref)
    yin = synth.white_complex((S.shape[0], k.shape[0]), 77)
    xa = to_np(plan.adjoint(to_dev(yin), Sd, dd))
    xa_ref = ndft.adjoint(yin, S, k, dcf)
    e_a = rel_l2(xa, xa_ref)
    xn = to_np(plan.normal(xd, Sd, dd))
    xn_ref = ndft.adjoint(y_ref, S, k, dcf)
    e_n = rel_l2(xn, xn_ref)
    say(f"   forward {e_f:.3e}  adjoint {e_a:.3e}  normal {e_n:.3e}  info={plan.info()}")
    return e_f, e_a, e_n


def test_tiny_radial_64(pnp):
    w = synth.config_tiny()
    x, S, k, _ = _case(w.n, w.L, w.traj.k, 1001)
    errs = _run_ops(pnp, (w.n, w.n), x, S, k, None, "64x64 L4 radial 16x128")
    assert max(errs) < TOL


def test_clinical_spiral_320_with_dcf(pnp):
    w = synth.config_clinical()
    dcf = synth.voronoi_dcf(w.traj, w.n)
    x, S, k, _ = _case(w.n, w.L, w.traj.k, 1002)
    errs = _run_ops(pnp, (w.n, w.n), x, S, k, dcf, "320x320 L16 spiral 32x400 + Voronoi DCF")
    assert max(errs) < TOL


@pytest.mark.parametrize("shape,L,M", [((48, 80), 5, 1000), ((8, 8), 1, 37), ((12, 20), 3, 333),
                                       ((96, 96), 6, 2049)])
def test_ragged_shapes_and_coils(pnp, shape, L, M):
    rng = np.random.default_rng(sum(shape) + L)
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    x = synth.white_complex(shape, 5)
    S = synth.white_complex((L,) + shape, 6)
    dcf = rng.uniform(0.2, 2.0, M).astype(np.float32)
    errs = _run_ops(pnp, shape, x, S, k, dcf, f"ragged {shape} L{L} M{M}")
    assert max(errs) < TOL


def test_samples_on_the_boundary_and_outside(pnp):
    """k = -pi, +pi, exact grid points and |k| > pi (the operator is 2*pi periodic)."""
    n = 32
    pts = [(-math.pi, -math.pi), (math.pi, 0.0), (0.0, 0.0), (-math.pi, math.pi / 2),
           (2 * math.pi / n, -4 * math.pi / n), (3.5, -3.9), (9.0, -7.0), (1e-7, -1e-7)]
    k = np.array(pts, dtype=np.float32)
    x = synth.white_complex((n, n), 8)
    S = synth.smaps2d(n, 2)
    errs = _run_ops(pnp, (n, n), x, S, k, None, "boundary samples")
    assert max(errs) < TOL


def test_full_cartesian_identity(pnp):
    """Full Cartesian sampling with SoS-1 maps: A^H A = I (up to the KB error)."""
    n = 32
    k = synth.cartesian2d(n)
    x = synth.white_complex((n, n), 9)
    S = synth.smaps2d(n, 4)
    plan = pnp.Plan(to_dev(k), (n, n))
    xn = to_np(plan.normal(to_dev(x), to_dev(S)))
    sos = (np.abs(S.astype(np.complex128)) ** 2).sum(0)
    assert rel_l2(xn, sos * x) < TOL


def test_adjoint_identity_on_gpu(pnp):
    n, L, M = 64, 4, 3000
    rng = np.random.default_rng(3)
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    x = synth.white_complex((n, n), 10)
    S = synth.smaps2d(n, L)
    yv = synth.white_complex((L, M), 11)
    plan = pnp.Plan(to_dev(k), (n, n))
    Sd = to_dev(S)
    Ax = to_np(plan.forward(to_dev(x), Sd)).astype(np.complex128)
    Ahy = to_np(plan.adjoint(to_dev(yv), Sd)).astype(np.complex128)
    lhs = np.vdot(Ax, yv.astype(np.complex128))
    rhs = np.vdot(x.astype(np.complex128), Ahy)
    assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_zero_input_gives_zero(pnp):
    w = synth.config_tiny()
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    import torch
    x = torch.zeros((w.n, w.n), dtype=torch.complex64, device="cuda")
    S = to_dev(synth.smaps2d(w.n, w.L))
    assert np.abs(to_np(plan.forward(x, S))).max() == 0.0
    assert np.abs(to_np(plan.normal(x, S))).max() == 0.0


def test_plan_rejects_nonfinite_trajectory(pnp):
    import torch
    k = torch.zeros((10, 2), dtype=torch.float32, device="cuda")
    k[3, 1] = float("nan")
    with pytest.raises(pnp.PnPError) as ei:
        pnp.Plan(k, (16, 16))
    assert ei.value.status == -6


def test_workspace_too_small_is_rejected(pnp):
    import ctypes as C
    import torch
    from paper_2411_01955_amd import _lib
    w = synth.config_tiny()
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    x = to_dev(synth.white_complex((w.n, w.n), 1))
    S = to_dev(synth.smaps2d(w.n, w.L))
    y = torch.empty((w.L, w.traj.k.shape[0]), dtype=torch.complex64, device="cuda")
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    st = _lib.load().pnp_forward(plan.handle, C.c_void_p(x.data_ptr()), C.c_void_p(S.data_ptr()), w.L,
                                 C.c_void_p(y.data_ptr()), C.c_void_p(ws.data_ptr()), 1024, None)
    assert st == -5


# ------------------------------------------------- Toeplitz normal operator
def _toep_case(pnp, shape, k, S, dcf, x, label, tol):
    plan = pnp.Plan(to_dev(k), shape)
    tp = pnp.Toeplitz(plan, to_dev(dcf) if dcf is not None else None)
    got = to_np(tp.normal(to_dev(x), to_dev(S)))
    ref = ndft.normal(x, S, k, dcf)
    e = rel_l2(got, ref)
    say(f"[toeplitz] {label}: rel {e:.3e}")
    assert e < tol
    return e


def test_toeplitz_tiny_radial(pnp):
    w = synth.config_tiny()
    x, _ = synth.phantom2d(w.n, 1001)
    _toep_case(pnp, (w.n, w.n), w.traj.k, synth.smaps2d(w.n, w.L), None, x, "64x64 L4 radial", 2e-6)


def test_toeplitz_clinical_spiral_dcf(pnp):
    w = synth.config_clinical()
    x, _ = synth.phantom2d(w.n, 1002)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    _toep_case(pnp, (w.n, w.n), w.traj.k, synth.smaps2d(w.n, w.L), dcf, x, "320x320 L16 spiral+DCF", 2e-6)


def test_toeplitz_ragged(pnp):
    rng = np.random.default_rng(12)
    shape, L, M = (96, 96), 5, 1777
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    k[:3] = [[-math.pi, -math.pi], [math.pi, 0.0], [0.0, 0.0]]
    dcf = rng.uniform(0.2, 2.0, M).astype(np.float32)
    x = synth.white_complex(shape, 13)
    S = synth.white_complex((L,) + shape, 14)
    _toep_case(pnp, shape, k, S, dcf, x, "96x96 L5 random+weights", 2e-6)


def test_toeplitz_rejects_unsupported_size(pnp):
    k = np.zeros((10, 2), np.float32)
    plan = pnp.Plan(to_dev(k), (48, 80))
    with pytest.raises(pnp.PnPError) as ei:
        pnp.Toeplitz(plan)
    assert ei.value.status == -3


# ------------------------------------------------- maximum sizes, rejections
@pytest.mark.parametrize("n,L,M,toeplitz", [(600, 2, 40000, False), (512, 4, 40000, True)])
def test_maximum_sizes_sampled(pnp, n, L, M, toeplitz):
    """The largest 2D image of the general passes (600^2: the 8-column strip
    of a 1200-point column fills 154 KB of LDS) and of the fused register-FFT
    and Toeplitz path (512^2): forward at sampled samples and adjoint at sampled
    pixels against the NDFT, the normal operator by its self-adjointness and,
    for 512^2, Toeplitz against gridded (both within the operator bar)."""
    rng = np.random.default_rng(n + L)
    k = rng.uniform(-math.pi, math.pi, (M, 2)).astype(np.float32)
    k[:2] = [[-math.pi, -math.pi], [0.0, 0.0]]
    dcf = rng.uniform(0.2, 2.0, M).astype(np.float32)
    x, _ = synth.phantom2d(n, 31)
    S = synth.smaps2d(n, L)
    plan = pnp.Plan(to_dev(k), (n, n))
    xd, Sd, dd = to_dev(x), to_dev(S), to_dev(dcf)
    idx = rng.choice(M, 48, replace=False)
    e_f = rel_l2(to_np(plan.forward(xd, Sd))[:, idx], ndft.forward_at(x, S, k, idx))
    yv = synth.white_complex((L, M), 32)
    pix = rng.choice(n * n, 48, replace=False)
    xa = to_np(plan.adjoint(to_dev(yv), Sd, dd))
    e_a = rel_l2(xa.reshape(-1)[pix], ndft.adjoint_at(yv, S, k, dcf, pix))
    normal = (lambda v: pnp.Toeplitz(plan, dd).normal(v, Sd)) if toeplitz else (lambda v: plan.normal(v, Sd, dd))
    x2 = synth.white_complex((n, n), 33)
    N1 = to_np(normal(xd)).astype(np.complex128)
    N2 = to_np(normal(to_dev(x2))).astype(np.complex128)
    lhs, rhs = np.vdot(x2.astype(np.complex128), N1), np.vdot(N2, x.astype(np.complex128))
    e_sa = abs(lhs - rhs) / abs(lhs)
    e_tg = rel_l2(N1, to_np(plan.normal(xd, Sd, dd)).astype(np.complex128)) if toeplitz else 0.0
    say(f"[ops] max size {n}x{n} L{L} M{M}: forward@48 {e_f:.2e} adjoint@48 {e_a:.2e} "
        f"self-adjoint {e_sa:.1e} Toeplitz vs gridded {e_tg:.2e}")
    assert max(e_f, e_a, e_tg) < TOL
    assert e_sa < 1e-5


def test_plan_rejects_bad_sizes(pnp):
    """Odd, too small or too large sides, grids with a prime factor above 5,
    four dimensions and an empty trajectory are refused (PNP_ERR_SHAPE), and
    a 2D grid too large for the LDS of its passes (PNP_ERR_UNSUPPORTED), when
    the plan is created."""
    import ctypes as C
    import torch
    from paper_2411_01955_amd import _lib
    k2 = torch.zeros((16, 2), dtype=torch.float32, device="cuda")
    for shape in [(15, 16), (16, 2), (2048, 16), (14, 16)]:
        with pytest.raises(pnp.PnPError) as ei:
            pnp.Plan(k2, shape)
        assert ei.value.status == -2, shape
    # a valid size whose column strip does not fit in LDS (2048-point columns)
    with pytest.raises(pnp.PnPError) as ei:
        pnp.Plan(k2, (1024, 1024))
    assert ei.value.status == -3
    h = C.c_void_p()
    for ndim, M in [(4, 16), (2, 0), (2, -3)]:
        shp = (C.c_int32 * 4)(16, 16, 16, 16)
        st = _lib.load().pnp_plan_create(C.byref(h), ndim, shp, M, C.c_void_p(k2.data_ptr()), None)
        assert st == -2, (ndim, M)
