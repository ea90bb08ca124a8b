"""Benchmark: annealed PnP-HQS on the clinical workload, one MI355X.

One *step* = one full annealed PnP-HQS reconstruction of a 320x320 slice
with 16 coils from a variable-density spiral (32 interleaves x 400 samples,
AF 8) with Voronoi density weighting: b0 = A^H D_w y, then 30 outer
iterations of (5-step CG proximal solve in the F-1 metric + Haar prior),
i.e. 180 applications of the normal operator A^H D_w A.  Inputs are seeded
synthetic phantoms already resident in HBM.

Printed JSON line:
* ``value``  HBM bandwidth of the whole step on the bytes its kernels move:
             the algorithmic (compulsory) bytes of every launch of the step
             (``kernel_bytes`` per launch x the step's launch counts, checked
             against a traced pass) / step time.  The Toeplitz operator the
             step runs moves ~138 MB per normal operator;
             ``value_b_alg_equivalent`` is the larger figure 180 * B_alg /
             step time, B_alg = the bytes of the gridded normal operator (x,
             coil maps twice, output, trajectory, DCF and four crossings of
             the oversampled coil grids), which the Toeplitz form avoids;
* ``roofline``  the dominant kernel's algorithmic bytes per launch over its
             mean launch time (HIP events around each launch, recorded on the
             kernel's stream over a second pass of the same steps), against
             8 TB/s; ``traffic`` from the committed rocprofv3 counter summary
             when it matches the current kernel sources; ``issue`` the same
             kernel against its FP32 VALU issue time (committed SQ counters
             of the same sources, 4 cycles per wave instruction on 1024
             SIMDs at 2.4 GHz) and its FP32 rate against 78.6 TFLOP/s (no
             packed FP32 instructions: the library is compiled without them);
* ``cpu_baseline``  the FP64 oracle (exact NDFT) timed on the host on one
             outer HQS iteration of the same slice (6 normal operators),
             scaled to the same unit;
* ``psnr_race``  slices/s to a fixed PSNR, learned (UNet, wavelet fallback)
             vs wavelet HQS: the target is the mean final PSNR of wavelet-HQS
             (30 iterations) over held-out phantoms, rounded down to 0.5 dB;
             per slice and method a logged run finds the first outer
             iteration k* that reaches it (30 if none does), and a timed run
             of exactly k* iterations gives seconds per slice;
* ``batched`` the 24-slice uneven table (n 256/320/384, 8/16/32 coils, AF
             4/8/16, radial and spiral, Voronoi DCF): the batched Toeplitz
             normal operator (one persistent launch per stage) against the
             sum of the slices' B_alg, and batched HQS (30 outer x 5 CG) in
             slices/s next to the same slices solved one after another;
* ``volume_3d`` the 128^3 / 32-coil / 4,096 x 256 kooshball volume: the 3D
             Toeplitz normal operator against B_alg, and HQS (20 outer x 5 CG)
             with the wavelet prior and with the UNet applied slice by slice;
* ``unet``   the denoiser's forward (320x320, batch 1 and 24) and training
             step (batch 10 x 128x128, forward + backward + Adam) in TFLOP/s
             and as a fraction of the 2.5 PFLOP/s dense BF16 MFMA peak;
* ``setup``  the once-per-trajectory and once-per-solve work of the clinical
             slice, outside the timed step: plan creation, the Toeplitz
             transfer function, the operator norm (100 power iterations), and
             the gridded forward and adjoint operators alone.

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
# hyperparameters tuned once on training phantoms (seeds 0..4): lambda*||N||, Haar threshold factor
LAM_TIMES_NORM = 1e4
KAPPA = 0.75
KAPPA_UNET = 1.0       # UNet conditioning level = kappa * sigma_k
RISE_TOL = 0.5         # wavelet fallback when the residual rises by more than 50%
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_clinical.json")
SQ_FILE = os.path.join(ROOT, "profiles", "sq_clinical.json")
# FP32 vector issue: a wave64 VALU instruction occupies a 16-lane SIMD for 4
# cycles; 256 CUs x 4 SIMDs at 2.4 GHz.  Packed FP32 instructions are not
# generated (the library is compiled without them), so the FP32 peak is 256 x 4 x 16 lanes x 2 (FMA) x
# 2.4 GHz = 78.6 TFLOP/s, half the packed figure.
VALU_CYCLES_PER_INST = 4
SIMDS = 1024
CLOCK_HZ = 2.4e9
FP32_PEAK_NONPACKED_TFLOPS = 78.6
KERNEL_SOURCES = ["paper_2411_01955_amd/csrc/nufft2d.hip", "paper_2411_01955_amd/csrc/fs_bodies.hpp",
                  "paper_2411_01955_amd/csrc/fft_lds.hpp", "paper_2411_01955_amd/csrc/fft_reg.hpp",
                  "paper_2411_01955_amd/csrc/common.hpp", "paper_2411_01955_amd/csrc/cg_scalars.hpp",
                  "paper_2411_01955_amd/csrc/plan.hip", "paper_2411_01955_amd/csrc/toeplitz.hip",
                  "paper_2411_01955_amd/csrc/solver.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def b_alg_normal(n, L, M, d=2):
    """Algorithmic bytes of one normal operator A^H D_w A (complex64 = 8 B):
    x + coil maps (forward and adjoint) + output + trajectory (twice) + DCF +
    4 crossings of the L oversampled (2n)^d grids."""
    N = n ** d
    G = (2 * n) ** d
    return 8 * N + 2 * 8 * L * N + 8 * N + 2 * 4 * d * M + 4 * M + 4 * 8 * L * G


def kernel_bytes(n, L, M, E, groups):
    """Algorithmic (compulsory) bytes per launch of each kernel of the fused
    2D operator (half-transformed grid mid[L][n][2n] crosses HBM twice per
    direction; per-sample plan data j0 16 B + weights 48 B; entries 4 B)."""
    N = n * n
    mid = 8 * L * n * 2 * n
    rec = 64 * E                      # packed per-entry taps and weights
    out = {
        "k_rows_fwd": 8 * N + 8 * L * N + mid,
        "k_cols_fwd_interp": mid + 8 * L * E + rec,
        "k_gather_entries": 8 * L * E + 8 * L * M + 8 * M,
        "k_cols_adj_spread": 8 * L * M + 4 * M + rec + mid,
        "k_rows_adj": mid + 8 * L * N + 8 * groups * N,
        "k_sum_groups": 8 * groups * N + 8 * N,
    }
    out["k_rows_fwd_fs"] = out["k_rows_fwd"]
    out["k_cols_fwd_fs"] = out["k_cols_fwd_interp"]
    out["k_cols_adj_fs"] = out["k_cols_adj_spread"]
    out["k_rows_adj_fs"] = out["k_rows_adj"]
    out["k_entry_values"] = 64 * E + 8 * L * E * 2 + 8 * M * 2 + 8 * L * E
    # parts of split strips added: no compulsory bytes beyond the spread's own
    # (its mid term counts every image row of every strip once)
    out["k_cols_adj_fin_fs"] = 0
    # Toeplitz column pass: mid in and out (image rows only) + the real transfer function once
    out["k_cols_toep_fs"] = 2 * mid + 4 * (2 * n) ** 2
    # CG vector kernels: w = c0 r + cg sum_g part_g (r, G partials in; w out),
    # the first step's (u, r, p, s) from (x, partials, b0), the last u update
    out["k_cg_dots"] = 8 * N * (2 + groups)
    out["k_cg_init"] = 8 * N * (2 + groups + 4)
    out["k_cg_final"] = 8 * N * 4
    # forward row pass with the CG update fused in: reads r, s, w, p, u and
    # writes r', s', p', u' (coil group 0) besides the plain pass's bytes
    out["k_rows_fwd_fs_cg"] = out["k_rows_fwd_fs"] - 8 * N + 8 * N * 9
    # the same with the step's inner products formed in the row passes: w is
    # rebuilt from r and the coil-group partial images (read instead of w),
    # and the adjoint row pass also reads r for its per-row sums of Re<part, r>
    out["k_rows_fwd_fs_cgf"] = out["k_rows_fwd_fs_cg"] + 8 * N * (groups - 1)
    # the first CG step's forward row pass with the CG start fused in: reads
    # b0 and the partial images of N x besides x, writes u, r, p, s (group 0)
    out["k_rows_fwd_fs_cgi"] = out["k_rows_fwd_fs"] + 8 * N * (1 + groups + 4)
    out["k_rows_adj_fs_dots"] = out["k_rows_adj_fs"] + 8 * N
    # Haar prior on the last CG update u + alpha (r + beta p): r, p, u in, x out
    out["k_haar_prior_cg"] = 8 * N * 4
    out["k_wnorm"] = 8 * L * M + 4 * M
    out["k_copy"] = 16 * N
    out["k_init_scalars"] = 0
    return out


def step_launches(n_out, n_cg, split_strips):
    """Launch counts of one wavelet-HQS solve on the Toeplitz operator (the
    timed step): per outer iteration N x (plain forward row pass) and n_cg
    CG steps (the first with the CG start r0 = gamma (b0 - N x) fused into
    its forward row pass, the rest with the CG update fused into it; the row
    passes of every step also form its inner products, so there is no
    reduction pass) and the prior on the last update; once per solve b0 = A^H D_w y (gridded adjoint: the spread,
    plus the pass that adds split strips' parts when the plan splits any),
    ||y||_w^2, x0 = b0 and the scalar reset."""
    return {"k_rows_fwd_fs": n_out, "k_rows_fwd_fs_cgi": n_out, "k_rows_fwd_fs_cgf": (n_cg - 1) * n_out,
            "k_cols_toep_fs": (1 + n_cg) * n_out, "k_rows_adj_fs": n_out + 1,
            "k_rows_adj_fs_dots": n_cg * n_out, "k_haar_prior_cg": n_out,
            "k_cols_adj_fs": 1, "k_cols_adj_fin_fs": 1 if split_strips else 0, "k_sum_groups": 1,
            "k_wnorm": 1, "k_copy": 1, "k_init_scalars": 1}


def toeplitz_normal_bytes(kb):
    """Algorithmic bytes of one Toeplitz normal operator alone (plain input)."""
    return kb["k_rows_fwd_fs"] + kb["k_cols_toep_fs"] + kb["k_rows_adj_fs"] + kb["k_sum_groups"]


def _kname(s: str) -> str:
    """Trace names of templated kernels carry '(name<K1, K2>)'."""
    s = s.strip("()")
    return s.split("<")[0]


UNET_LEVEL = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "e3a": 2, "e3b": 2, "ba": 3, "bb": 3, "up3": 3,
              "d3a": 2, "d3b": 2, "up2": 2, "d2a": 1, "d2b": 1, "up1": 1, "d1a": 0, "d1b": 0, "out": 0}


def unet_flops(layers, B, H, W, backward=False):
    """Multiply-add FLOPs (x2) of the UNet's contractions for a batch of B
    images H x W (real input channels; transposed convs per input pixel and
    tap).  The backward pass is the input- and weight-gradient contractions
    (twice the forward, without the first layer's input gradient)."""
    fwd = 0
    first = 0
    for l in layers:
        P = B * (H >> UNET_LEVEL[l["name"]]) * (W >> UNET_LEVEL[l["name"]])
        f = 2 * P * l["taps"] * l["cin"] * l["cout"]
        fwd += f
        if l["name"] == "e1a":
            first = f
    return fwd + (2 * fwd - first if backward else 0)


def psnr_roi(xr, x, roi):
    e = np.abs(xr)[roi] - np.abs(x)[roi]
    return 20 * math.log10(np.abs(x)[roi].max() / math.sqrt(np.mean(e ** 2)))


def psnr_race(pnp, torch, plan, toep, Sd, dd, w, S, nrm, n_slices):
    """Slices/s to a fixed PSNR, learned vs wavelet HQS, on held-out phantoms."""
    import synth
    n, L = w.n, w.L
    M = w.traj.k.shape[0]
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    lam = LAM_TIMES_NORM / nrm
    wav = pnp.WaveletPrior(0, KAPPA)
    net = pnp.trained_unet()
    lrn = pnp.UNetPrior(net, (n, n), KAPPA_UNET, fallback=wav)
    methods = {"wavelet": wav, "learned": lrn}
    slices = []
    for i in range(n_slices):
        seed = synth.SEED_HELDOUT + i
        x, roi = synth.phantom2d(n, seed)
        y = plan.forward(torch.from_numpy(x).cuda(), Sd)
        y += torch.from_numpy(synth.complex_noise((L, M), synth.noise_variance(x, S), synth.SEED_NOISE + seed)).cuda()
        slices.append((x, roi, y))

    def solve(prior, y, sigmas, x0=None):
        return pnp.hqs_solve(plan, y, Sd, dd, prior, sigmas, lam, "f1", w.n_cg, opnorm=nrm, x0=x0, toeplitz=toep,
                             rise_tol=RISE_TOL)[0]

    # logged runs: one-iteration solves chained through x0 are the same iterates
    curves = {m: [] for m in methods}
    for x, roi, y in slices:
        for m, prior in methods.items():
            xk, c = None, []
            for k in range(len(sig)):
                xk = solve(prior, y, sig[k:k + 1], xk).clone()
                c.append(psnr_roi(xk.cpu().numpy(), x, roi))
            curves[m].append(c)
    final = {m: float(np.mean([c[-1] for c in curves[m]])) for m in methods}
    target = math.floor(final["wavelet"] * 2) / 2
    out = {"target_psnr_db": target, "slices": n_slices, "held_out_seeds": f"{synth.SEED_HELDOUT}.."
           f"{synth.SEED_HELDOUT + n_slices - 1}", "final_psnr_db": {m: round(v, 2) for m, v in final.items()}}
    for m, prior in methods.items():
        ks = [next((k + 1 for k, v in enumerate(c) if v >= target), len(sig)) for c in curves[m]]
        reached = sum(1 for c in curves[m] if max(c) >= target)
        solve(prior, slices[0][2], sig[:2])       # warm-up
        torch.cuda.synchronize()
        secs = []
        for (x, roi, y), k in zip(slices, ks):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            solve(prior, y, sig[:k])
            b.record()
            torch.cuda.synchronize()
            secs.append(a.elapsed_time(b) / 1e3)
        out[m] = {"slices_per_s": round(1.0 / float(np.mean(secs)), 2), "mean_outer_iterations": round(float(np.mean(ks)), 2),
                  "max_outer_iterations": int(max(ks)),
                  "reached_target": f"{reached}/{n_slices}", "ms_per_slice": round(1e3 * float(np.mean(secs)), 3)}
    out["learned_over_wavelet"] = round(out["learned"]["slices_per_s"] / out["wavelet"]["slices_per_s"], 2)
    out["learned_prior"] = f"UNet (kappa {KAPPA_UNET}) with wavelet fallback (rise_tol {RISE_TOL})"
    return out


def setup_times(pnp, torch, kt, shape, xd, Sd, dd, y, time_op):
    """Plan creation, Toeplitz transfer function and operator norm (median of
    3, each synchronised), and the gridded A and A^H alone (median of the
    event-timed repetitions)."""
    def once(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3, r

    plan_ms, tp_ms, nrm_ms = [], [], []
    for _ in range(3):
        t, pl = once(lambda: pnp.Plan(kt, shape))
        plan_ms.append(t)
        t, tp = once(lambda: pnp.Toeplitz(pl, dd))
        tp_ms.append(t)
        nrm_ms.append(once(lambda: pl.opnorm(Sd, dd, iters=100, seed=1))[0])
        tp.close()
        pl.close()
    pl = pnp.Plan(kt, shape)
    ybuf = torch.empty_like(y)
    xbuf = torch.empty_like(xd)
    fwd_us = time_op(lambda: pl.forward(xd, Sd, out=ybuf))[0]
    adj_us = time_op(lambda: pl.adjoint(y, Sd, dd, out=xbuf))[0]
    pl.close()
    med = lambda v: round(float(np.median(v)), 3)
    return {"plan_create_ms": med(plan_ms), "toeplitz_transfer_function_ms": med(tp_ms),
            "opnorm_100_iterations_ms": med(nrm_ms), "forward_us": round(fwd_us, 2),
            "adjoint_us": round(adj_us, 2)}


def pgd_fista(pnp, torch, plan, toep, Sd, dd, w, S, nrm, seed, b_alg):
    """PnP-PGD (Id, F-1; wavelet prior on the annealed sigma schedule) and
    FISTA-Wavelet on the clinical slice, 30 iterations each, gamma = 1/||N||:
    time per solve, normal operators per second and final PSNR.  The FISTA
    weight is picked once on a training phantom (seed 0) from a small grid."""
    import synth
    n, L = w.n, w.L
    M = w.traj.k.shape[0]
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    gamma = 1.0 / nrm
    wav = pnp.WaveletPrior(0, KAPPA)

    def data(sd):
        x, roi = synth.phantom2d(n, sd)
        y = plan.forward(torch.from_numpy(x).cuda(), Sd)
        y += torch.from_numpy(synth.complex_noise((L, M), synth.noise_variance(x, S), synth.SEED_NOISE + sd)).cuda()
        return x, roi, y

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    xt, rt, yt = data(0)
    scale = float(plan.adjoint(yt, Sd, dd).abs().max())
    best = None
    for rel in (1e-3, 3e-3, 1e-2, 3e-2):
        lam = rel * scale * nrm
        xr = pnp.fista_wavelet(plan, yt, Sd, dd, lam, gamma, w.n_out, toeplitz=toep)
        p = psnr_roi(xr.cpu().numpy(), xt, rt)
        if best is None or p > best[1]:
            best = (rel, p)
    x, roi, y = data(seed)
    out = {"iterations": w.n_out, "gamma_times_norm": 1.0}
    runs = {
        "pgd_id": (lambda: pnp.pgd_solve(plan, y, Sd, dd, wav, sig, gamma, "id", opnorm=nrm, toeplitz=toep), 1),
        "pgd_f1": (lambda: pnp.pgd_solve(plan, y, Sd, dd, wav, sig, gamma, "f1", opnorm=nrm, toeplitz=toep), 2),
        "fista_wavelet": (lambda: pnp.fista_wavelet(plan, y, Sd, dd, best[0] * scale * nrm, gamma, w.n_out,
                                                    toeplitz=toep), 1),
    }
    for name, (fn, ops) in runs.items():
        xr, sec = timed(fn)
        n_ops = ops * w.n_out
        out[name] = {"ms_per_solve": round(sec * 1e3, 3), "normal_ops": n_ops,
                     "GBps": round(n_ops * b_alg / sec / 1e9, 1), "psnr_db": round(psnr_roi(xr.cpu().numpy(), x, roi), 2)}
    out["fista_wavelet"]["lam_rel_to_max_b0"] = best[0]
    return out


def batched_c4(pnp, torch, reps=10):
    """The 24-slice table through the batched path vs one slice at a time."""
    import synth
    w = synth.config_clinical()
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    slices, b_alg = [], 0
    for sl in synth.batched_slice_table():
        i, n, L, tr = sl["index"], sl["n"], sl["L"], sl["traj"]
        M = tr.k.shape[0]
        x, _ = synth.phantom2d(n, synth.SEED_PHANTOM + i)
        S = synth.smaps2d(n, L)
        dcf = synth.voronoi_dcf(tr, n)
        plan = pnp.Plan(torch.from_numpy(tr.k).cuda(), (n, n))
        Sd, dd = torch.from_numpy(S).cuda(), torch.from_numpy(dcf).cuda()
        y = plan.forward(torch.from_numpy(x).cuda(), Sd)
        y += torch.from_numpy(synth.complex_noise((L, M), synth.noise_variance(x, S), synth.SEED_NOISE + i)).cuda()
        nrm = plan.opnorm(Sd, dd, iters=60, seed=1)
        slices.append(dict(plan=plan, toeplitz=pnp.Toeplitz(plan, dd), y=y, smaps=Sd, dcf=dd, opnorm=nrm,
                           lam=LAM_TIMES_NORM / nrm))
        b_alg += b_alg_normal(n, L, M)
    batch = pnp.Batch(slices)
    xs = [torch.from_numpy(synth.white_complex(d["plan"].shape, 5)).cuda() for d in slices]
    outs = [torch.empty_like(x) for x in xs]

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n / 1e3

    t_op = timed(lambda: batch.normal(xs, outs), reps)
    t_op_seq = timed(lambda: [d["toeplitz"].normal(x, d["smaps"], out=o) for d, x, o in zip(slices, xs, outs)], reps)
    wav = pnp.WaveletPrior(0, KAPPA)
    t_hqs = timed(lambda: batch.hqs_solve(wav, sig, "f1", w.n_cg), 2)
    t_seq = timed(lambda: [pnp.hqs_solve(d["plan"], d["y"], d["smaps"], d["dcf"], wav, sig, d["lam"], "f1", w.n_cg,
                                         opnorm=d["opnorm"], toeplitz=d["toeplitz"], out=o)
                           for d, o in zip(slices, outs)], 2)
    lrn = pnp.UNetPrior(pnp.trained_unet(), (320, 320), KAPPA_UNET)
    k_l = 4
    t_lrn = timed(lambda: batch.hqs_solve(lrn, sig[:k_l], "f1", w.n_cg), 2)
    n_ops = w.n_out * (1 + w.n_cg)
    return {"slices": len(slices), "b_alg_bytes_per_normal_op": b_alg,
            "normal_op_ms": round(t_op * 1e3, 3), "normal_op_GBps": round(b_alg / t_op / 1e9, 1),
            "normal_op_frac_of_hbm": round(b_alg / t_op / 1e9 / HBM_PEAK_GBPS, 4),
            "normal_op_one_by_one_ms": round(t_op_seq * 1e3, 3),
            "hqs_wavelet_ms": round(t_hqs * 1e3, 2), "hqs_wavelet_slices_per_s": round(len(slices) / t_hqs, 1),
            "hqs_wavelet_GBps": round(n_ops * b_alg / t_hqs / 1e9, 1),
            "hqs_wavelet_one_by_one_slices_per_s": round(len(slices) / t_seq, 1),
            "hqs_learned_outer": k_l, "hqs_learned_ms": round(t_lrn * 1e3, 2),
            "hqs_learned_slices_per_s": round(len(slices) / t_lrn, 1)}


def volume_3d(pnp, torch, n_out=None):
    """The 128^3 / 32-coil / 4,096 x 256 kooshball workload: Toeplitz normal
    operator against its B_alg, and one annealed HQS volume (wavelet prior,
    and the UNet applied slice by slice) -- data from the GPU forward operator."""
    import synth
    w = synth.config_3d()
    n, L = w.n, w.L
    k = w.traj.k
    M = k.shape[0]
    x, _ = synth.phantom3d(n, synth.SEED_PHANTOM)
    S = synth.smaps3d(n, L)
    dcf = synth.radial3d_dcf(w.traj, n)
    plan = pnp.Plan(torch.from_numpy(k).cuda(), (n, n, n))
    Sd, dd = torch.from_numpy(S).cuda(), torch.from_numpy(dcf).cuda()
    xd = torch.from_numpy(x).cuda()
    y = plan.forward(xd, Sd)
    y += torch.from_numpy(synth.complex_noise((L, M), synth.noise_variance(x, S), synth.SEED_NOISE)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    toep = pnp.Toeplitz(plan, dd)      # exact FP64 transfer function (waits for the stream)
    progress("3D plan and transfer function built")
    t_toep = time.perf_counter() - t0
    nrm = plan.opnorm(Sd, dd, iters=30, seed=1)
    out = torch.empty_like(xd)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps / 1e3

    B = b_alg_normal(n, L, M, d=3)
    t_op = timed(lambda: toep.normal(xd, Sd, out=out), 5)
    yt = torch.empty_like(y)
    t_fwd = timed(lambda: plan.forward(xd, Sd, out=yt), 3)
    del yt
    t_adj = timed(lambda: plan.adjoint(y, Sd, dd, out=out), 3)   # b0's gridded adjoint (type-1 spread)
    n_out = n_out or w.n_out
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)[:n_out]
    lam = LAM_TIMES_NORM / nrm
    wav = pnp.WaveletPrior(0, KAPPA)
    t_hqs = timed(lambda: pnp.hqs_solve(plan, y, Sd, dd, wav, sig, lam, "f1", w.n_cg, opnorm=nrm, out=out,
                                        toeplitz=toep), 1)
    lrn = pnp.UNetPrior(pnp.trained_unet(), (n, n, n), KAPPA_UNET, fallback=wav)
    t_lrn = timed(lambda: pnp.hqs_solve(plan, y, Sd, dd, lrn, sig, lam, "f1", w.n_cg, opnorm=nrm, out=out,
                                        toeplitz=toep, rise_tol=RISE_TOL), 1)
    n_ops = n_out * (1 + w.n_cg)
    return {"workload": w.name, "b_alg_bytes_per_normal_op": B, "toeplitz_normal_op_ms": round(t_op * 1e3, 3),
            "toeplitz_normal_op_GBps": round(B / t_op / 1e9, 1),
            "toeplitz_normal_op_frac_of_hbm": round(B / t_op / 1e9 / HBM_PEAK_GBPS, 4),
            "forward_ms": round(t_fwd * 1e3, 3), "adjoint_ms": round(t_adj * 1e3, 3),
            "hqs_outer": n_out, "hqs_wavelet_s_per_volume": round(t_hqs, 3),
            "hqs_wavelet_GBps": round(n_ops * B / t_hqs / 1e9, 1),
            "hqs_learned_slicewise_s_per_volume": round(t_lrn, 3),
            "toeplitz_transfer_function_s": round(t_toep, 3)}


def unet_rates(pnp, torch):
    """Forward and training-step throughput of the denoiser (inputs resident)."""
    import synth
    layers = pnp.unet_layers()
    net = pnp.trained_unet()
    res = {}

    def timed(fn, reps):
        for _ in range(3):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps / 1e3

    for B in (1, 24):
        u = torch.from_numpy(synth.white_complex((B, 320, 320), 3) * 0.5).cuda()
        sg = torch.full((B,), 0.05, dtype=torch.float32, device="cuda")
        o = torch.empty_like(u)
        t = timed(lambda: net.forward(u, sg, out=o), 20 if B == 1 else 5)
        fl = unet_flops(layers, B, 320, 320)
        res[f"fwd_320_b{B}"] = {"ms": round(t * 1e3, 3), "gflop": round(fl / 1e9, 2),
                                "tflops": round(fl / t / 1e12, 1),
                                "mfma_util": round(fl / t / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)}
    trainer = pnp.UNet(net.get("params"))
    u = torch.from_numpy(synth.white_complex((10, 128, 128), 4) * 0.5).cuda()
    tg = (u * 0.9).contiguous()
    sg = torch.full((10,), 0.05, dtype=torch.float32, device="cuda")

    def train_step():
        trainer.forward(u, sg, train=True)
        trainer.backward(u, tg)
        trainer.adam_step(0.0)          # lr 0: the step runs, the weights stay
    t = timed(train_step, 20)
    fl = unet_flops(layers, 10, 128, 128, backward=True)
    res["train_step_b10_128"] = {"ms": round(t * 1e3, 3), "gflop": round(fl / 1e9, 2),
                                 "tflops": round(fl / t / 1e12, 1),
                                 "mfma_util": round(fl / t / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)}
    # Neighbor2Neighbor step: f(x) on the full patches, f(g1(x)) forward and
    # backward on the half-size sub-images, Adam
    codes = torch.randint(0, 8, (10, 64, 64), dtype=torch.uint8, device="cuda")

    def n2n_step():
        trainer.n2n_backward(u, codes, 2.0)
        trainer.adam_step(0.0)
    t = timed(n2n_step, 20)
    fl = unet_flops(layers, 10, 128, 128) + unet_flops(layers, 10, 64, 64, backward=True)
    res["n2n_step_b10_128"] = {"ms": round(t * 1e3, 3), "gflop": round(fl / 1e9, 2),
                               "tflops": round(fl / t / 1e12, 1),
                               "mfma_util": round(fl / t / 1e12 / MFMA_BF16_PEAK_TFLOPS, 4)}
    res["peak_tflops"] = MFMA_BF16_PEAK_TFLOPS
    return res


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(w, x, S, dcf, y, step_bytes):
    """Oracle (exact NDFT, numpy/OpenBLAS FP64) on one outer HQS iteration of
    the same slice (1 + n_cg normal operators, the prior and the residual
    operator) with all host threads, and one exact normal operator with one
    thread; both extrapolated to a whole slice (30 outer iterations) and
    reported in the step's unit: the step's bytes / the oracle's time per
    slice (the GPU/CPU ratio of `value` is then the ratio of slice times)."""
    from oracle import ndft, solver, wavelet
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    k = w.traj.k
    normal = lambda v: ndft.normal(v, S, k, dcf)
    b0 = ndft.adjoint(y, S, k, dcf)
    t0 = time.perf_counter()
    solver.hqs(b0, normal, [w.sigma0], 1.0, "f1", w.n_cg,
               lambda u, s: wavelet.wavelet_denoise(u, KAPPA * s), 17.0)
    dt = time.perf_counter() - t0
    per_slice = dt * w.n_out
    out = {"value": round(step_bytes / per_slice / 1e9, 4), "unit": "GB/s", "cores": int(cores), "kind": "oracle",
           "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
           "sample": f"one outer HQS iteration (1+{w.n_cg} CG normal operators + prior + residual operator) of "
                     f"the 320x320/16-coil spiral slice, exact FP64 NDFT, {dt:.1f} s with {cores} threads; "
                     f"x {w.n_out} = {per_slice:.0f} s per slice; value = the step's bytes / that time",
           "seconds_per_slice_extrapolated": round(per_slice, 1)}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            normal(x)
            d1 = time.perf_counter() - t0
        ops = w.n_out * (1 + w.n_cg + 1)
        out["one_thread"] = {"normal_op_s": round(d1, 2), "seconds_per_slice_extrapolated": round(d1 * ops, 1),
                             "value": round(step_bytes / (d1 * ops) / 1e9, 5),
                             "sample": f"one exact normal operator with 1 thread, x {ops} operators per slice"}
    return out


_T0 = time.perf_counter()


def progress(msg):
    """One line per finished leg on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg} ({time.perf_counter() - _T0:.0f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device copy (counter calibration for rocprofv3)")
    ap.add_argument("--seed", type=int, default=1002)
    ap.add_argument("--reps", type=int, default=200,
                    help="back-to-back repetitions when timing the normal operators alone")
    ap.add_argument("--psnr-slices", type=int, default=100,
                    help="held-out phantoms of the learned-vs-wavelet PSNR race (0: skip)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 24-slice batched measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the 128^3 measurement")
    ap.add_argument("--no-pgd", action="store_true", help="skip the PnP-PGD / FISTA-Wavelet measurement")
    ap.add_argument("--row-coils", default="",
                    help="FWD,ADJ coils per row-pass workgroup (2, 4 or 8) instead of the autotuner's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): slices are independent "
              "and a slice's coils only meet in the image sum, so the workload would shard across GPUs by "
              "slice or by coil group with one image all-reduce per normal operator, but no multi-GPU "
              "path is built or measured.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2411_01955_amd as pnp

    dev = torch.device("cuda:0")
    w = synth.config_clinical()
    n, L = w.n, w.L
    k = w.traj.k
    M = k.shape[0]
    x_true, roi = synth.phantom2d(n, args.seed)
    S = synth.smaps2d(n, L)
    dcf = synth.voronoi_dcf(w.traj, n)
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)

    kt = torch.from_numpy(k).to(dev)
    xd = torch.from_numpy(x_true).to(dev)
    Sd = torch.from_numpy(S).to(dev)
    dd = torch.from_numpy(dcf).to(dev)
    plan = pnp.Plan(kt, (n, n))
    info = plan.info()
    # simulated acquisition (Sec. 4.1): y = A x + e, nu = 1e-4 max sum_l |S_l x|^2
    y = plan.forward(xd, Sd)
    nu = synth.noise_variance(x_true, S)
    y += torch.from_numpy(synth.complex_noise((L, M), nu, synth.SEED_NOISE + args.seed)).to(dev)
    nrm = plan.opnorm(Sd, dd, iters=100, seed=1)
    lam = LAM_TIMES_NORM / nrm
    prior = pnp.WaveletPrior(0, KAPPA)
    out = torch.empty((n, n), dtype=torch.complex64, device=dev)
    ws, _ = plan.workspace(L, "hqs")
    toep = pnp.Toeplitz(plan, dd)      # transfer function built once per (trajectory, DCF)
    if args.row_coils:
        # fixed launch shape (profiling runs: a profiler's per-launch overhead
        # hides the differences the tuner times)
        fwd_rc, adj_rc = (int(v) for v in args.row_coils.split(","))
        plan.row_coils_pair = (fwd_rc, adj_rc)
        tuning = {"row_coils": adj_rc, "row_coils_fwd": fwd_rc, "fixed": True}
    else:
        tuning = plan.autotune(Sd, dd, toeplitz=toep)   # coils per row-pass workgroup, timed on this GPU

    def step():
        pnp.hqs_solve(plan, y, Sd, dd, prior, sig, lam, "f1", w.n_cg, opnorm=nrm, out=out, toeplitz=toep)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    step_ms = [a.elapsed_time(b) for a, b in ev]
    n_normal = w.n_out * (1 + w.n_cg)
    B = b_alg_normal(n, L, M)
    groups = -(-L // plan.row_coils)
    kb = kernel_bytes(n, L, M, info["entries"], groups)
    launches_model = step_launches(w.n_out, w.n_cg, plan.spread[0] > 0)
    step_bytes = sum(kb[k] * c for k, c in launches_model.items())
    value = step_bytes / (ms / 1e3) / 1e9
    value_b_alg = n_normal * B / (ms / 1e3) / 1e9

    # quality of the reconstruction (outside the timed region)
    xr = out.cpu().numpy()
    from_mag = np.abs(xr)
    err = from_mag[roi] - np.abs(x_true)[roi]
    psnr = 20 * math.log10(np.abs(x_true)[roi].max() / math.sqrt(np.mean(err ** 2)))

    # normal operator alone, back to back: gridded and Toeplitz-embedded
    tmp = torch.empty_like(xd)

    def time_op(fn, reps=max(100, args.reps)):
        """Median (p10, p90) of `reps` back-to-back repetitions, each between
        two HIP events on the launch stream, in microseconds."""
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        us = np.array([a.elapsed_time(b) * 1e3 for a, b in evs])
        return float(np.median(us)), float(np.percentile(us, 10)), float(np.percentile(us, 90))

    gridded_us, gridded_p10, gridded_p90 = time_op(lambda: plan.normal(xd, Sd, dd, out=tmp))
    normal_us, normal_p10, normal_p90 = time_op(lambda: toep.normal(xd, Sd, out=tmp))
    toep_bytes = toeplitz_normal_bytes(kb)

    # traced pass: per-kernel durations with HIP events on the launch stream
    pnp.trace_enable(True)
    pnp.trace_read()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    tr = {}
    for kname, (c, t) in pnp.trace_read().items():
        c0, t0 = tr.get(_kname(kname), (0, 0.0))
        tr[_kname(kname)] = (c0 + c, t0 + t)
    pnp.trace_enable(False)
    # the byte model's launch counts against the traced ones (the plain and
    # CG-fused row passes share their kernels' names)
    counted = {kname: c // args.steps for kname, (c, t) in tr.items()}
    model = dict(launches_model)
    model["k_rows_fwd_fs"] = (model.pop("k_rows_fwd_fs") + model.pop("k_rows_fwd_fs_cgi")
                              + model.pop("k_rows_fwd_fs_cgf"))
    model["k_rows_adj_fs"] = model.pop("k_rows_adj_fs") + model.pop("k_rows_adj_fs_dots")
    launch_check = {k: [model.get(k, 0), counted.get(k, 0)] for k in sorted(set(model) | set(counted))
                    if model.get(k, 0) != counted.get(k, 0)}
    dom = max((kname for kname in tr if kname in kb), key=lambda kname: tr[kname][1])
    launches, tot_ms = tr[dom]
    avg_s = tot_ms / launches / 1e3
    achieved = kb[dom] / avg_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tf = json.load(f)
        ent = tf.get("kernels", {}).get(dom)
        if ent and tf.get("source_hash") == kernel_source_hash():
            traffic = ent.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": kb[dom], "avg_launch_us": round(avg_s * 1e6, 2)}
    # the same kernel against its FP32 issue bound, from the committed SQ
    # instruction counters of the same sources (null once they changed)
    roofline["issue"] = None
    if os.path.exists(SQ_FILE):
        with open(SQ_FILE) as f:
            sq = json.load(f)
        ent = sq.get("kernels", {}).get(dom)
        if ent and sq.get("source_hash") == kernel_source_hash():
            issue_s = ent["valu_per_launch"] * VALU_CYCLES_PER_INST / SIMDS / CLOCK_HZ
            roofline["issue"] = {
                "valu_instructions_per_launch": ent["valu_per_launch"],
                "valu_issue_us": round(issue_s * 1e6, 2),
                "frac": round(issue_s / avg_s, 4),
                "fp32_flops_per_launch": ent["fp32_flops_per_launch"],
                "fp32_tflops": round(ent["fp32_flops_per_launch"] / avg_s / 1e12, 2),
                "fp32_peak_nonpacked_tflops": FP32_PEAK_NONPACKED_TFLOPS}
    kernel_table = {kname: {"launches": c, "avg_us": round(t / c * 1e3, 2),
                            "share": round(t / sum(v[1] for v in tr.values()), 4)}
                    for kname, (c, t) in sorted(tr.items(), key=lambda kv: -kv[1][1])}

    if args.calib_copy:
        a = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    progress("timed HQS step and operators done")
    race = psnr_race(pnp, torch, plan, toep, Sd, dd, w, S, nrm, args.psnr_slices) if args.psnr_slices > 0 else None
    progress("PSNR race done")
    others = None if args.no_pgd else pgd_fista(pnp, torch, plan, toep, Sd, dd, w, S, nrm, args.seed, B)
    progress("PGD / FISTA done")
    # coil sensitivity estimate from the k-space centre of the same data (20 x 20 Hamming window)
    pnp.estimate_smaps(plan, y, dd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        pnp.estimate_smaps(plan, y, dd)
    torch.cuda.synchronize()
    smaps_ms = (time.perf_counter() - t0) * 1e2
    setup = setup_times(pnp, torch, kt, (n, n), xd, Sd, dd, y, time_op)
    progress("coil maps and set-up times done")
    unet = unet_rates(pnp, torch)
    progress("UNet rates done")
    batched = None if args.no_batched else batched_c4(pnp, torch)
    progress("batched slices done")
    vol3d = None if args.no_3d else volume_3d(pnp, torch)
    progress("3D volume done")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, x_true, S, dcf, y.cpu().numpy(), step_bytes)
        progress("CPU oracle baseline done")

    line = {
        "metric": "NUFFT A^H A GB/s; slices/s to fixed PSNR, learned vs wavelet HQS",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "coils": L, "samples": M, "outer": w.n_out, "cg": w.n_cg,
                   "prior": "haar", "precond": "f1", "dcf": "voronoi", "normal_ops_per_step": n_normal,
                   "value_bytes": "algorithmic bytes of every kernel launch of the step (Toeplitz normal "
                                  "operator, CG vectors, prior, b0)",
                   "step_bytes": step_bytes, "b_alg_bytes": B},
        "value_frac_of_hbm": round(value / HBM_PEAK_GBPS, 4),
        "value_b_alg_equivalent": {"GBps": round(value_b_alg, 1), "frac_of_hbm": round(value_b_alg / HBM_PEAK_GBPS, 4),
                                   "meaning": "180 x B_alg of the gridded normal operator / step time: more "
                                              "bytes than the Toeplitz step moves"},
        "step_ms_p10_p50_p90": [round(float(np.percentile(step_ms, q)), 4) for q in (10, 50, 90)],
        "launch_model_mismatch": launch_check,
        "slices_per_s": round(1e3 / ms, 3),
        "psnr_db": round(psnr, 3),
        "normal_op_us": round(normal_us, 2),
        "normal_op_us_p10_p90": [round(normal_p10, 2), round(normal_p90, 2)],
        "normal_op_bytes": toep_bytes,
        "normal_op_GBps": round(toep_bytes / (normal_us * 1e-6) / 1e9, 1),
        "normal_op_frac_of_hbm": round(toep_bytes / (normal_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4),
        "normal_op_b_alg_equivalent_GBps": round(B / (normal_us * 1e-6) / 1e9, 1),
        "normal_op_variant": "toeplitz (exact PSF transfer function; used inside the HQS step); median of "
                             f"{max(100, args.reps)} event-timed repetitions",
        "gridded_normal_op_us": round(gridded_us, 2),
        "gridded_normal_op_us_p10_p90": [round(gridded_p10, 2), round(gridded_p90, 2)],
        "gridded_normal_op_GBps_b_alg": round(B / (gridded_us * 1e-6) / 1e9, 1),
        "roofline": roofline,
        "autotune": tuning,
        "psnr_race": race,
        "pgd_fista": others,
        "smaps_estimate_ms": round(smaps_ms, 3),
        "setup": setup,
        "batched": batched,
        "volume_3d": vol3d,
        "unet": unet,
        "kernels": kernel_table,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
