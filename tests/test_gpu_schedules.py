"""Oracle parity at the schedules the benchmark times (Sec. 3.3-3.4).

The annealed HQS is an iteration, so its final image is compared with the
oracle's after the full schedule, not after a few steps.  The oracle runs
are stored under tests/golden/ (written by tests/golden/make_golden.py,
which calls only the oracle); the data y are recomputed here from the same
seeds with the oracle's exact forward operator.  Bar: relative L2 <= 1e-4
on the final image.

* the timed clinical step itself: 320^2, 16 coils, spiral 32 x 400,
  Voronoi DCF, lambda*||N|| = 1e4, kappa = 0.75, F-1, 30 outer x 5 CG, on
  the Toeplitz normal operator the step uses (and on the gridded one);
* a 64^3 / 2-coil kooshball volume over the full 20-outer schedule on the
  3D Toeplitz operator with its exact transfer function;
* three uneven slices (256/320/384, 8/16/32 coils, radial and spiral, AF 16)
  through the batched solver, each against its own oracle HQS;
* the 384^2 / 32-coil operators at full size on sampled outputs.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ndft
from tests.golden import make_golden
from tests.gpu_util import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BAR = 1e-4


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


@pytest.mark.parametrize("toeplitz", [True, False])
def test_bench_step_matches_golden(pnp, toeplitz):
    meta = _load("hqs_bench_seed1002")
    x_ref = np.load(os.path.join(GOLDEN, "hqs_bench_seed1002.npy"))
    w, x, roi, S, dcf, y = make_golden.clinical_inputs(meta["seed"])
    say(f"[schedule] clinical bench step, toeplitz={toeplitz}: data ready")
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    dd, Sd = to_dev(dcf), to_dev(S)
    tp = pnp.Toeplitz(plan, dd) if toeplitz else None
    nrm = meta["opnorm"]
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    xg, _ = pnp.hqs_solve(plan, to_dev(y), Sd, dd, pnp.WaveletPrior(0, meta["kappa"]), sig,
                          meta["lam_times_norm"] / nrm, meta["precond"], w.n_cg, opnorm=nrm, toeplitz=tp)
    e = rel_l2(to_np(xg), x_ref)
    say(f"[schedule] clinical 30 x 5, lambda*||N|| = 1e4, toeplitz={toeplitz}: final image rel {e:.2e}")
    assert e < BAR


def test_3d_full_schedule_matches_golden(pnp):
    meta = _load("hqs_vol3d")
    x_ref = np.load(os.path.join(GOLDEN, "hqs_vol3d.npy"))
    tr, x, roi, S, dcf, y = make_golden.vol3d_inputs()
    n = meta["n"]
    say(f"[schedule] 3D {n}^3 L={meta['L']} M={tr.k.shape[0]}: data ready")
    plan = pnp.Plan(to_dev(tr.k), (n, n, n))
    dd = to_dev(dcf)
    tp = pnp.Toeplitz(plan, dd)
    nrm = meta["opnorm"]
    sig = synth.geometric_sigmas(0.1, 0.005, meta["n_out"])
    xg, _ = pnp.hqs_solve(plan, to_dev(y), to_dev(S), dd, pnp.WaveletPrior(0, meta["kappa"]), sig,
                          meta["lam_times_norm"] / nrm, meta["precond"], meta["n_cg"], opnorm=nrm, toeplitz=tp)
    e = rel_l2(to_np(xg), x_ref)
    say(f"[schedule] 3D {n}^3 20 x 5 (Toeplitz, exact transfer function): final image rel {e:.2e}")
    assert e < BAR


def test_batch3_matches_golden(pnp):
    meta = _load("hqs_batch3")
    c = meta["hqs"]
    slices, refs = [], []
    for i, sm in enumerate(meta["slices"]):
        tr, x, roi, S, dcf, y = make_golden.batch3_inputs(i)
        plan = pnp.Plan(to_dev(tr.k), (sm["n"], sm["n"]))
        dd = to_dev(dcf)
        slices.append(dict(plan=plan, toeplitz=pnp.Toeplitz(plan, dd), y=to_dev(y), smaps=to_dev(S), dcf=dd,
                           opnorm=sm["opnorm"], lam=c["lam_times_norm"] / sm["opnorm"]))
        refs.append(np.load(os.path.join(GOLDEN, f"hqs_batch3_{i}.npy")))
        say(f"[schedule] batch slice {i}: {sm['n']}^2 L={sm['L']} {sm['kind']} M={sm['M']} ready")
    batch = pnp.Batch(slices)
    sig = synth.geometric_sigmas(0.1, 0.005, c["n_out"])
    outs, _ = batch.hqs_solve(pnp.WaveletPrior(0, c["kappa"]), sig, c["precond"], c["n_cg"])
    errs = [rel_l2(to_np(o), r) for o, r in zip(outs, refs)]
    say(f"[schedule] batched 3 uneven slices, 30 x 5: final image rel {['%.2e' % e for e in errs]}")
    assert max(errs) < BAR


def test_384_operators_at_full_size_sampled(pnp):
    """384^2, 32 coils, radial AF 4 (M = 36,864): the forward at 48 random
    samples and the adjoint at 48 random pixels against the exact NDFT (each
    output entry exact on its own), and the Toeplitz normal operator against
    the gridded one."""
    n, L = 384, 32
    tr = synth.uneven_slice_traj(n, 4, True)
    k = tr.k
    M = k.shape[0]
    x, _ = synth.phantom2d(n, 1201)
    S = synth.smaps2d(n, L)
    dcf = synth.voronoi_dcf(tr, n)
    plan = pnp.Plan(to_dev(k), (n, n))
    Sd, dd, xd = to_dev(S), to_dev(dcf), to_dev(x)
    y = to_np(plan.forward(xd, Sd))
    rng = np.random.default_rng(12)
    idx = rng.choice(M, 48, replace=False)
    e_f = rel_l2(y[:, idx], ndft.forward_at(x, S, k, idx))
    yv = synth.white_complex((L, M), 13)
    xa = to_np(plan.adjoint(to_dev(yv), Sd, dd))
    vox = rng.choice(n * n, 48, replace=False)
    e_a = rel_l2(xa.reshape(-1)[vox], ndft.adjoint_at(yv, S, k, dcf, vox))
    Ng = to_np(plan.normal(xd, Sd, dd))
    Nt = to_np(pnp.Toeplitz(plan, dd).normal(xd, Sd))
    e_tg = rel_l2(Nt, Ng)
    say(f"[schedule] 384^2 L=32 M={M}: forward@48 {e_f:.2e}, adjoint@48 {e_a:.2e}, Toeplitz vs gridded {e_tg:.2e}")
    assert max(e_f, e_a, e_tg) < 2e-5
