"""Kernel tracing: every launch of a traced call is counted under its kernel
name, the durations are the kernels' own (their sum stays below the wall
time of the calls), tracing off records nothing, and a read clears the
counts."""
import time

import numpy as np
import pytest

import synth
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


def _kname(s):
    return s.strip("()").split("<")[0]


def test_trace_counts_and_durations(pnp):
    import torch
    w = synth.config_clinical()
    x, _ = synth.phantom2d(w.n, 3)
    S = to_dev(synth.smaps2d(w.n, w.L))
    dcf = to_dev(synth.voronoi_dcf(w.traj, w.n))
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    tp = pnp.Toeplitz(plan, dcf)
    xd = to_dev(x)
    out = torch.empty_like(xd)
    for _ in range(3):
        tp.normal(xd, S, out=out)
    torch.cuda.synchronize()
    pnp.trace_read()                          # drop anything recorded so far
    pnp.trace_enable(True)
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        tp.normal(xd, S, out=out)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    tr = pnp.trace_read()
    pnp.trace_enable(False)
    names = {_kname(k): v for k, v in tr.items()}
    say(f"[trace] {reps} Toeplitz normal ops, wall {wall_ms:.3f} ms: "
        + ", ".join(f"{k} {c}x {t / c * 1e3:.2f} us" for k, (c, t) in names.items()))
    for k in ("k_rows_fwd_fs", "k_cols_toep_fs", "k_rows_adj_fs"):
        assert k in names and names[k][0] == reps
    assert all(t > 0 for _, t in tr.values())
    assert sum(t for _, t in tr.values()) < wall_ms
    # off: nothing recorded; a read clears
    tp.normal(xd, S, out=out)
    torch.cuda.synchronize()
    assert pnp.trace_read() == {}
    assert np.isfinite(out.abs().max().item())
