"""Autotuned launch shape: the operators agree with the oracle for every
coils-per-workgroup choice (2, 4, 8) of the forward and the adjoint row
pass, alike and mixed, and the tuner picks a pair, records it in its
JSON-lines cache and reapplies it from there without timing."""
import json

import numpy as np
import pytest

import synth
from oracle import ndft
from tests.gpu_util import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


@pytest.mark.parametrize("rc", [2, 4, 8, (8, 2), (2, 8), (4, 8)])
def test_operators_match_oracle_for_every_row_coils(pnp, rc):
    w = synth.config_tiny()
    x, _ = synth.phantom2d(w.n, 5)
    S = synth.smaps2d(w.n, 6)                # 6 coils: a ragged last group for 4 and 8
    k = w.traj.k
    dcf = np.random.default_rng(7).uniform(0.5, 1.5, k.shape[0]).astype(np.float32)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    if isinstance(rc, tuple):
        plan.row_coils_pair = rc
        assert plan.row_coils_pair == rc and plan.row_coils == rc[1]
    else:
        plan.row_coils = rc
        assert plan.row_coils == rc and plan.row_coils_pair == (rc, rc)
    xd, Sd, dd = to_dev(x), to_dev(S), to_dev(dcf)
    ref = ndft.normal(x, S, k, dcf)
    e_g = rel_l2(to_np(plan.normal(xd, Sd, dd)), ref)
    e_t = rel_l2(to_np(pnp.Toeplitz(plan, dd).normal(xd, Sd)), ref)
    y = synth.white_complex((6, k.shape[0]), 8)
    e_a = rel_l2(to_np(plan.adjoint(to_dev(y), Sd, dd)), ndft.adjoint(y, S, k, dcf))
    say(f"[tune] row_coils={rc}: gridded {e_g:.2e} toeplitz {e_t:.2e} adjoint {e_a:.2e}")
    assert max(e_g, e_a) < 2e-5 and e_t < 2e-6


@pytest.mark.parametrize("rc", [(4, 4), (2, 8), (8, 4)])
def test_toeplitz_hqs_with_ragged_coil_groups(pnp, rc):
    """Toeplitz HQS with 6 coils, whose CG inner products are summed per coil
    group by the adjoint row pass (three groups of 2, two of 4 with a partial
    last one, or one partial group of 8), against the oracle's HQS."""
    import dataclasses
    from oracle import solver, wavelet
    w = dataclasses.replace(synth.config_tiny(), L=6, n_out=6)
    x, _ = synth.phantom2d(w.n, 4)
    S = synth.smaps2d(w.n, w.L)
    k = w.traj.k
    dcf = np.random.default_rng(9).uniform(0.5, 1.5, k.shape[0]).astype(np.float32)
    nu = synth.noise_variance(x, S)
    y = (ndft.forward(x, S, k) + synth.complex_noise((w.L, k.shape[0]), nu, synth.SEED_NOISE + 4)).astype(np.complex64)
    normal = lambda v: ndft.normal(v, S, k, dcf)
    # the norm only parameterises the problem and is handed to both sides
    Ln, _ = solver.opnorm(normal, (w.n, w.n), tol=1e-8, maxit=300)
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    lam = 30000.0 / Ln
    x_ref = solver.hqs(ndft.adjoint(y, S, k, dcf), normal, sig, lam, "f1", w.n_cg,
                       lambda u, s: wavelet.wavelet_denoise(u, 0.5 * s), Ln)
    plan = pnp.Plan(to_dev(k), (w.n, w.n))
    plan.row_coils_pair = rc
    dd = to_dev(dcf)
    xg, _ = pnp.hqs_solve(plan, to_dev(y), to_dev(S), dd, pnp.WaveletPrior(0, 0.5), sig, lam, "f1", w.n_cg,
                          opnorm=Ln, toeplitz=pnp.Toeplitz(plan, dd))
    e = rel_l2(to_np(xg), x_ref)
    say(f"[tune] Toeplitz HQS, 6 coils, row_coils={rc}: image rel {e:.3e}")
    assert e < 1e-4


@pytest.fixture(scope="module")
def clinical_adjoint_ref():
    w = synth.config_clinical()
    S = synth.smaps2d(w.n, w.L)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    y = synth.white_complex((w.L, w.traj.k.shape[0]), 21)
    return w, S, dcf, y, ndft.adjoint(y, S, w.traj.k, dcf)


@pytest.mark.parametrize("split", [0, 1, 2, 3])
@pytest.mark.parametrize("dense_min", [128, 512])
def test_adjoint_matches_oracle_for_every_spread_setting(pnp, clinical_adjoint_ref, split, dense_min):
    """The clinical spiral's heavy strips (the k-space centre) split into 0
    to several parts, and the dense-block threshold: the adjoint against the
    exact NDFT for each setting, and bit-identical to the unsplit spread
    where no row block changes hands between the shared and the per-wave
    form (same dense threshold, so the per-block sums are the same)."""
    w, S, dcf, y, ref = clinical_adjoint_ref
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    plan.spread = (split, dense_min)
    assert plan.spread == (split, dense_min)
    Sd, dd, yd = to_dev(S), to_dev(dcf), to_dev(y)
    got = to_np(plan.adjoint(yd, Sd, dd))
    e = rel_l2(got, ref)
    plan.spread = (0, dense_min)
    base = to_np(plan.adjoint(yd, Sd, dd))
    say(f"[tune] spread split={split} dense_min={dense_min}: adjoint {e:.2e}, "
        f"max |split - unsplit| = {np.abs(got - base).max():.2e}")
    assert e < 2e-5
    assert rel_l2(got, base) < 1e-6


def test_autotune_and_cache(pnp, tmp_path):
    w = synth.config_clinical()
    S = to_dev(synth.smaps2d(w.n, w.L))
    dcf = to_dev(synth.voronoi_dcf(w.traj, w.n))
    cache = str(tmp_path / "tune.jsonl")
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    tp = pnp.Toeplitz(plan, dcf)
    r1 = plan.autotune(S, dcf, toeplitz=tp, cache=cache)
    say(f"[tune] clinical Toeplitz: {r1}")
    pair = (r1["row_coils_fwd"], r1["row_coils"])
    assert set(pair) <= {2, 4, 8} and not r1["from_cache"]
    assert all(t > 0 for t in r1["time_us"] + r1["time_fwd_us"])
    assert plan.row_coils_pair == pair
    assert plan.spread == (r1["spread_split"], r1["spread_dense_min"])
    assert r1["spread_split"] in (0, 1, 2, 3) and r1["spread_dense_min"] in (128, 256, 512)
    assert all(t > 0 for t in r1["time_spread_us"])
    ts = r1["time_spread_us"]
    chosen = ts[3 * r1["spread_split"] + (128, 256, 512).index(r1["spread_dense_min"])]
    assert chosen <= ts[3]                               # never slower than the default (split 1, 128)
    t = dict(zip((2, 4, 8), r1["time_us"]))
    tf = dict(zip((2, 4, 8), r1["time_fwd_us"]))
    assert t[pair[1]] <= t[4] and tf[pair[0]] <= tf[4]   # never slower than the default
    lines = [json.loads(l) for l in open(cache)]
    assert len(lines) == 1 and (lines[0]["row_coils_fwd"], lines[0]["row_coils"]) == pair
    # a second plan on the same trajectory takes the cached choice
    plan2 = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    plan2.row_coils_pair = tuple(2 if v != 2 else 8 for v in pair)
    plan2.spread = (0, 512)
    r2 = plan2.autotune(S, dcf, toeplitz=pnp.Toeplitz(plan2, dcf), cache=cache)
    assert r2["from_cache"] and (r2["row_coils_fwd"], r2["row_coils"]) == pair == plan2.row_coils_pair
    assert plan2.spread == (r1["spread_split"], r1["spread_dense_min"])
    # the gridded operator is a different key
    r3 = plan2.autotune(S, dcf, cache=cache)
    assert not r3["from_cache"]
    assert len(open(cache).readlines()) == 2


def test_tuned_plan_gives_the_same_hqs(pnp):
    w = synth.config_clinical()
    x, _ = synth.phantom2d(w.n, 9)
    S = synth.smaps2d(w.n, w.L)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    Sd, dd = to_dev(S), to_dev(dcf)
    y = plan.forward(to_dev(x), Sd)
    tp = pnp.Toeplitz(plan, dd)
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)[:3]
    outs = {}
    for rc in (2, 4, 8):
        plan.row_coils = rc
        xr, _ = pnp.hqs_solve(plan, y, Sd, dd, pnp.WaveletPrior(0, 0.75), sig, 1e4 / 17.45, "f1", 5,
                              opnorm=17.45, toeplitz=tp)
        outs[rc] = to_np(xr)
    e = max(rel_l2(outs[2], outs[4]), rel_l2(outs[8], outs[4]))
    say(f"[tune] HQS with 2/4/8 coils per workgroup: max rel difference {e:.2e}")
    assert e < 1e-5


def test_row_coils_rejects_other_values(pnp):
    w = synth.config_tiny()
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    with pytest.raises(pnp.PnPError):
        plan.row_coils = 3
    with pytest.raises(pnp.PnPError):
        plan.row_coils_pair = (4, 6)
    with pytest.raises(pnp.PnPError):
        plan.row_coils_pair = (16, 4)
    assert plan.row_coils_pair == (4, 4)
