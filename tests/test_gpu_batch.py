"""Batched uneven slices: every slice of the batched launches must
equal its single-slice computation (rel L2 <= 1e-5), over the 24-slice table
(n in {256, 320, 384}, L in {8, 16, 32}, AF 4/8/16, radial and spiral).
The single-slice path is itself pinned to the FP64 oracle in the operator
and solver tests; one batched slice is also compared with the oracle here.

Density weights are seeded U(0.5, 1.5) (the batching does not depend on
their meaning; Voronoi cells for 24 trajectories take ~16 s on the host)."""
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


def _slices(pnp, count=24, lam_times_norm=1e4):
    out = []
    for sl in synth.batched_slice_table(count):
        i, n, L = sl["index"], sl["n"], sl["L"]
        k = sl["traj"].k
        M = k.shape[0]
        x, roi = synth.phantom2d(n, synth.SEED_PHANTOM + i)
        S = synth.smaps2d(n, L)
        dcf = np.random.default_rng(300 + i).uniform(0.5, 1.5, M).astype(np.float32)
        plan = pnp.Plan(to_dev(k), (n, n))
        Sd, dd = to_dev(S), to_dev(dcf)
        tp = pnp.Toeplitz(plan, dd)
        y = plan.forward(to_dev(x), Sd)
        y += to_dev(synth.complex_noise((L, M), synth.noise_variance(x, S), synth.SEED_NOISE + i))
        nrm = plan.opnorm(Sd, dd, iters=60, seed=1)
        out.append(dict(plan=plan, toeplitz=tp, y=y, smaps=Sd, dcf=dd, opnorm=nrm, lam=lam_times_norm / nrm,
                        x=x, roi=roi, k=k, S=S, dcf_np=dcf, n=n, L=L))
    return out


@pytest.fixture(scope="module")
def slices(pnp):
    return _slices(pnp)


def test_batched_normal_equals_single(pnp, slices):
    batch = pnp.Batch(slices)
    xs = [to_dev(synth.white_complex((d["n"], d["n"]), 50 + j)) for j, d in enumerate(slices)]
    outs = batch.normal(xs)
    worst = 0.0
    for j, (d, x, o) in enumerate(zip(slices, xs, outs)):
        ref = d["toeplitz"].normal(x, d["smaps"])
        e = rel_l2(to_np(o), to_np(ref))
        worst = max(worst, e)
    say(f"[batch] normal operator, 24 slices: worst rel {worst:.2e}")
    assert worst < 1e-5


def test_batched_slice_matches_oracle(pnp, slices):
    """The smallest-M slice of the table through the batched operator vs the exact NDFT."""
    j = min(range(len(slices)), key=lambda i: slices[i]["k"].shape[0] * slices[i]["L"])
    d = slices[j]
    batch = pnp.Batch([d])
    x = synth.white_complex((d["n"], d["n"]), 71)
    got = to_np(batch.normal([to_dev(x)])[0])
    ref = ndft.normal(x, d["S"], d["k"], d["dcf_np"])
    e = rel_l2(got, ref)
    say(f"[batch] slice {j} (n={d['n']}, L={d['L']}, M={d['k'].shape[0]}) vs NDFT: rel {e:.2e}")
    assert e < 2e-6


def test_batched_hqs_wavelet_equals_single(pnp, slices):
    w = synth.config_clinical()
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)[:4]
    prior = pnp.WaveletPrior(0, 0.75)
    batch = pnp.Batch(slices)
    outs, rho = batch.hqs_solve(prior, sig, "f1", 5, report=True)
    worst, worst_rho = 0.0, 0.0
    for j, d in enumerate(slices):
        ref, rep = pnp.hqs_solve(d["plan"], d["y"], d["smaps"], d["dcf"], prior, sig, d["lam"], "f1", 5,
                                 opnorm=d["opnorm"], toeplitz=d["toeplitz"], report=True)
        worst = max(worst, rel_l2(to_np(outs[j]), to_np(ref)))
        yw2 = float((d["dcf_np"] * np.abs(to_np(d["y"]).astype(np.complex128)) ** 2).sum())
        worst_rho = max(worst_rho, max(abs(a - b) for a, b in zip(rho[j], rep["rho"])) / yw2)
    say(f"[batch] wavelet HQS, 24 slices x 4 outer: worst image rel {worst:.2e}, rho {worst_rho:.2e}")
    assert worst < 1e-5
    assert worst_rho < 1e-6


def test_batched_hqs_unet_equals_single(pnp, slices):
    sub = slices[:6]                       # two slices of each size
    w = synth.config_clinical()
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)[:2]
    net = pnp.trained_unet()
    batch = pnp.Batch(sub)
    prior_b = pnp.UNetPrior(net, (sub[0]["n"], sub[0]["n"]), 1.0)
    outs, _ = batch.hqs_solve(prior_b, sig, "f1", 5)
    worst = 0.0
    for j, d in enumerate(sub):
        pr = pnp.UNetPrior(net, (d["n"], d["n"]), 1.0)
        ref, _ = pnp.hqs_solve(d["plan"], d["y"], d["smaps"], d["dcf"], pr, sig, d["lam"], "f1", 5,
                               opnorm=d["opnorm"], toeplitz=d["toeplitz"])
        worst = max(worst, rel_l2(to_np(outs[j]), to_np(ref)))
    say(f"[batch] UNet HQS, 6 slices x 2 outer: worst image rel {worst:.2e}")
    assert worst < 1e-5


def test_batch_rejects_unsupported_size(pnp):
    """A non-square slice (its Toeplitz embedding exists) is refused."""
    import torch
    k = synth.radial2d(8, 128).k
    plan = pnp.Plan(to_dev(k), (64, 128))
    S = to_dev(synth.white_complex((2, 64, 128), 3))
    tp = pnp.Toeplitz(plan)
    y = torch.zeros((2, k.shape[0]), dtype=torch.complex64, device="cuda")
    with pytest.raises(pnp.PnPError) as ei:
        pnp.Batch([dict(plan=plan, toeplitz=tp, y=y, smaps=S, dcf=None, opnorm=1.0, lam=1.0)])
    assert ei.value.status == -3
