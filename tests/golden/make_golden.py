"""Write the stored expected values under tests/golden/ (oracle only).

Every value here is computed by the FP64 oracle from the seeded synthetic
inputs; nothing comes from the GPU library.

    python -m tests.golden.make_golden opnorm     # ~15 min on 8 cores
    python -m tests.golden.make_golden hqs        # ~5 min on 8 cores

* ``opnorm_clinical.json``: ||A^H D_w A||_2 of the 320x320 / 16-coil /
  spiral 32x400 / Voronoi-DCF operator, by Lanczos on the exact NDFT normal
  operator (the largest eigenvalue; alpha = 1/norm normalises the
  preconditioners of Sec. 3.4).
* ``hqs_clinical_seed1002.npy``: the oracle's final annealed PnP-HQS image
  (exact NDFT, F-1 preconditioner, 30 outer x 5 CG, Haar prior) for
  phantom seed 1002, stored as complex128.
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


def clinical_inputs(seed: int):
    w = synth.config_clinical()
    x, roi = synth.phantom2d(w.n, seed)
    S = synth.smaps2d(w.n, w.L)
    dcf = synth.voronoi_dcf(w.traj, w.n)
    nu = synth.noise_variance(x, S)
    y = ndft.forward(x, S, w.traj.k) + synth.complex_noise((w.L, w.traj.k.shape[0]), nu,
                                                           synth.SEED_NOISE + seed)
    return w, x, roi, S, dcf, y.astype(np.complex64)


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
    t = time.time()

    def prior(u, s):
        print(f"  sigma {s:.4f}  t={time.time() - t:.0f}s", flush=True)
        return wavelet.wavelet_denoise(u, cfg["kappa"] * s)

    xh = solver.hqs(b0, normal, sig, cfg["lam_times_norm"] / Ln, cfg["precond"], w.n_cg, prior, Ln)
    np.save(os.path.join(HERE, f"hqs_clinical_seed{cfg['seed']}.npy"), xh)


if __name__ == "__main__":
    what = sys.argv[1:] or ["opnorm", "hqs"]
    if "opnorm" in what:
        make_opnorm()
    if "hqs" in what:
        make_hqs()
