"""Write the stored expected values under tests/golden/ (oracle only).

Every value here is computed by the FP64 oracle from the seeded synthetic
inputs; nothing comes from the GPU library.  Each item prints its progress.

    python -m tests.golden.make_golden opnorm     # ~15 min on 8 cores
    python -m tests.golden.make_golden hqs        # ~5 min on 8 cores
    python -m tests.golden.make_golden bench      # ~5 min
    python -m tests.golden.make_golden vol3d      # ~20 min
    python -m tests.golden.make_golden batch3     # ~20 min

* ``opnorm_clinical.json``: ||A^H D_w A||_2 of the 320x320 / 16-coil /
  spiral 32x400 / Voronoi-DCF operator, by Lanczos on the exact NDFT normal
  operator (the largest eigenvalue; alpha = 1/norm normalises the
  preconditioners of Sec. 3.4).
* ``hqs_clinical_seed1002.npy``: the oracle's final annealed PnP-HQS image
  (exact NDFT, F-1 preconditioner, 30 outer x 5 CG, Haar prior,
  lambda*||N|| = 30, kappa = 1) for phantom seed 1002, complex128.
* ``hqs_bench_seed1002.npy`` (+ ``.json``): the same slice with the
  hyperparameters of the timed benchmark step (lambda*||N|| = 1e4,
  kappa = 0.75, F-1, 30 outer x 5 CG, Voronoi DCF), complex64.
* ``hqs_vol3d.npy`` (+ ``.json``): a 64^3 / 2-coil / 256 x 128 kooshball
  volume (N/M = 8) with the radial 3D density weights, the full 20-outer x 5-CG
  annealed schedule, lambda*||N|| = 1e4, kappa = 0.75, F-1, complex64.
* ``hqs_batch3_<i>.npy`` (+ ``hqs_batch3.json``): three uneven slices
  (256^2 / 8 coils / radial, 320^2 / 16 coils / spiral, 384^2 / 32 coils /
  spiral, all AF 16 by the uneven-table rule, Voronoi DCF), each solved by
  the oracle's HQS with the benchmark hyperparameters, complex64.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import ndft, solver, wavelet  # noqa: E402

HQS_CLINICAL = {"seed": 1002, "precond": "f1", "lam_times_norm": 30.0, "kappa": 1.0}
# the benchmark step's settings (tuned once on training phantoms 0..4)
HQS_BENCH = {"seed": 1002, "precond": "f1", "lam_times_norm": 1e4, "kappa": 0.75}
VOL_3D = {"n": 64, "L": 2, "spokes": 256, "S": 128, "seed": 1005, "precond": "f1", "lam_times_norm": 1e4,
          "kappa": 0.75, "n_out": 20, "n_cg": 5}
BATCH3 = [{"n": 256, "L": 8, "af": 16, "radial": True, "seed": 1101},
          {"n": 320, "L": 16, "af": 16, "radial": False, "seed": 1102},
          {"n": 384, "L": 32, "af": 16, "radial": False, "seed": 1103}]
BATCH3_HQS = {"precond": "f1", "lam_times_norm": 1e4, "kappa": 0.75, "n_out": 30, "n_cg": 5}


def clinical_inputs(seed: int):
    w = synth.config_clinical()
    x, roi = synth.phantom2d(w.n, seed)
    S = synth.smaps2d(w.n, w.L)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    nu = synth.noise_variance(x, S)
    y = ndft.forward(x, S, w.traj.k) + synth.complex_noise((w.L, w.traj.k.shape[0]), nu,
                                                           synth.SEED_NOISE + seed)
    return w, x, roi, S, dcf, y.astype(np.complex64)


def vol3d_inputs():
    c = VOL_3D
    tr = synth.kooshball3d(c["spokes"], c["S"])
    x, roi = synth.phantom3d(c["n"], c["seed"])
    S = synth.smaps3d(c["n"], c["L"])
    dcf = synth.radial3d_dcf(tr, c["n"])
    nu = synth.noise_variance(x, S)
    y = ndft.forward(x, S, tr.k) + synth.complex_noise((c["L"], tr.k.shape[0]), nu, synth.SEED_NOISE + c["seed"])
    return tr, x, roi, S, dcf, y.astype(np.complex64)


def batch3_inputs(i: int):
    c = BATCH3[i]
    tr = synth.uneven_slice_traj(c["n"], c["af"], c["radial"])
    x, roi = synth.phantom2d(c["n"], c["seed"])
    S = synth.smaps2d(c["n"], c["L"])
    dcf = synth.voronoi_dcf(tr, c["n"])
    nu = synth.noise_variance(x, S)
    y = ndft.forward(x, S, tr.k) + synth.complex_noise((c["L"], tr.k.shape[0]), nu, synth.SEED_NOISE + c["seed"])
    return tr, x, roi, S, dcf, y.astype(np.complex64)


def _progress(t0, label):
    def prior_cb(s):
        print(f"  {label} sigma {s:.4f}  t={time.time() - t0:.0f}s", flush=True)
    return prior_cb


def _oracle_hqs(b0, normal, sigmas, lam_times_norm, norm, precond, n_cg, kappa, label, levels=None):
    t0 = time.time()
    cb = _progress(t0, label)

    def prior(u, s):
        cb(s)
        return wavelet.wavelet_denoise(u, kappa * s, levels)
    return solver.hqs(b0, normal, sigmas, lam_times_norm / norm, precond, n_cg, prior, norm)


def _lanczos(normal, shape, label):
    t = time.time()
    calls = [0]

    def counted(v):
        calls[0] += 1
        if calls[0] % 10 == 0:
            print(f"  {label} Lanczos: {calls[0]} operator calls, t={time.time() - t:.0f}s", flush=True)
        return normal(v)
    val = solver.opnorm_lanczos(counted, shape, tol=1e-8)
    print(f"  {label} norm {val:.6f} ({calls[0]} calls, {time.time() - t:.0f}s)", flush=True)
    return val


def make_opnorm():
    w = synth.config_clinical()
    S = synth.smaps2d(w.n, w.L)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    t = time.time()
    L = solver.opnorm_lanczos(lambda v: ndft.normal(v, S, w.traj.k, dcf), (w.n, w.n), tol=1e-8)
    out = {"workload": w.name, "opnorm": L, "method": "Lanczos (scipy eigsh, tol 1e-8) on oracle.ndft",
           "seconds": time.time() - t}
    with open(os.path.join(HERE, "opnorm_clinical.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


def load_opnorm() -> float:
    with open(os.path.join(HERE, "opnorm_clinical.json")) as f:
        return float(json.load(f)["opnorm"])


def make_hqs():
    cfg = HQS_CLINICAL
    w, x, roi, S, dcf, y = clinical_inputs(cfg["seed"])
    Ln = load_opnorm()
    k = w.traj.k
    normal = lambda v: ndft.normal(v, S, k, dcf)
    b0 = ndft.adjoint(y, S, k, dcf)
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    xh = _oracle_hqs(b0, normal, sig, cfg["lam_times_norm"], Ln, cfg["precond"], w.n_cg, cfg["kappa"], "clinical")
    np.save(os.path.join(HERE, f"hqs_clinical_seed{cfg['seed']}.npy"), xh)


def make_bench():
    cfg = HQS_BENCH
    w, x, roi, S, dcf, y = clinical_inputs(cfg["seed"])
    Ln = load_opnorm()
    k = w.traj.k
    normal = lambda v: ndft.normal(v, S, k, dcf)
    b0 = ndft.adjoint(y, S, k, dcf)
    sig = synth.geometric_sigmas(w.sigma0, w.sigma_end, w.n_out)
    t = time.time()
    xh = _oracle_hqs(b0, normal, sig, cfg["lam_times_norm"], Ln, cfg["precond"], w.n_cg, cfg["kappa"], "bench")
    np.save(os.path.join(HERE, f"hqs_bench_seed{cfg['seed']}.npy"), xh.astype(np.complex64))
    meta = dict(cfg, workload=w.name, n_out=w.n_out, n_cg=w.n_cg, opnorm=Ln, seconds=time.time() - t,
                note="oracle HQS (exact NDFT normal operator), image stored as complex64")
    with open(os.path.join(HERE, f"hqs_bench_seed{cfg['seed']}.json"), "w") as f:
        json.dump(meta, f, indent=1)


def make_vol3d():
    c = VOL_3D
    tr, x, roi, S, dcf, y = vol3d_inputs()
    shape = (c["n"],) * 3
    normal = lambda v: ndft.normal(v, S, tr.k, dcf)
    Ln = _lanczos(normal, shape, "3d")
    b0 = ndft.adjoint(y, S, tr.k, dcf)
    sig = synth.geometric_sigmas(0.1, 0.005, c["n_out"])
    t = time.time()
    xh = _oracle_hqs(b0, normal, sig, c["lam_times_norm"], Ln, c["precond"], c["n_cg"], c["kappa"], "3d")
    np.save(os.path.join(HERE, "hqs_vol3d.npy"), xh.astype(np.complex64))
    with open(os.path.join(HERE, "hqs_vol3d.json"), "w") as f:
        json.dump(dict(c, opnorm=Ln, seconds=time.time() - t, M=int(tr.k.shape[0]),
                       note="oracle HQS (exact NDFT), radial 3D density weights, complex64 image"), f, indent=1)


def make_batch3():
    c = BATCH3_HQS
    meta = {"hqs": c, "slices": []}
    for i, sl in enumerate(BATCH3):
        tr, x, roi, S, dcf, y = batch3_inputs(i)
        shape = (sl["n"], sl["n"])
        normal = lambda v, S=S, k=tr.k, dcf=dcf: ndft.normal(v, S, k, dcf)
        Ln = _lanczos(normal, shape, f"batch3[{i}]")
        b0 = ndft.adjoint(y, S, tr.k, dcf)
        sig = synth.geometric_sigmas(0.1, 0.005, c["n_out"])
        t = time.time()
        xh = _oracle_hqs(b0, normal, sig, c["lam_times_norm"], Ln, c["precond"], c["n_cg"], c["kappa"],
                         f"batch3[{i}]")
        np.save(os.path.join(HERE, f"hqs_batch3_{i}.npy"), xh.astype(np.complex64))
        meta["slices"].append(dict(sl, M=int(tr.k.shape[0]), kind=tr.kind, opnorm=Ln, seconds=time.time() - t))
        with open(os.path.join(HERE, "hqs_batch3.json"), "w") as f:
            json.dump(meta, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1:] or ["opnorm", "hqs"]
    makers = {"opnorm": make_opnorm, "hqs": make_hqs, "bench": make_bench, "vol3d": make_vol3d,
              "batch3": make_batch3}
    for name in what:
        makers[name]()
