"""The Toeplitz normal operator's entry point that allocates nothing
(pnp_normal_toeplitz_noalloc, static per-device scratch) against the
workspace entry point pnp_normal_toeplitz on the same inputs: bit-identical
results on two calls in a row, the second on a smaller problem (so stale
scratch from the first call must not leak into it), the result checked
against the exact NDFT as well, and requests beyond the static scratch
refused before anything runs."""
import ctypes as C

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


def _case(pnp, n, L, traj, dcf, seed):
    import torch
    plan = pnp.Plan(to_dev(traj.k), (n, n))
    dd = to_dev(dcf) if dcf is not None else None
    tp = pnp.Toeplitz(plan, dd)
    x = synth.white_complex((n, n), seed)
    S = synth.smaps2d(n, L)
    xd, Sd = to_dev(x), to_dev(S)
    ref = tp.normal(xd, Sd)
    out = torch.full((n, n), float("nan"), dtype=torch.complex64, device=xd.device)
    tp.normal_noalloc(xd, Sd, out)
    a, b = to_np(out), to_np(ref)
    e_ndft = rel_l2(a, ndft.normal(x, S, traj.k, dcf))
    say(f"[noalloc] n={n} L={L} M={traj.k.shape[0]}: bit-identical {np.array_equal(a, b)}, vs NDFT {e_ndft:.2e}")
    return a, b, e_ndft


def test_noalloc_matches_workspace_entry_point_twice(pnp):
    nb = C.c_size_t()
    assert pnp.load().pnp_noalloc_scratch_bytes(C.byref(nb)) == 0
    assert nb.value == 64 << 20
    w = synth.config_clinical()
    a, b, e = _case(pnp, w.n, w.L, w.traj, synth.voronoi_dcf(w.traj, w.n), 3)
    assert np.array_equal(a, b)
    assert e < 2e-5
    t = synth.config_tiny()
    a, b, e = _case(pnp, t.n, t.L, t.traj, None, 4)
    assert np.array_equal(a, b)
    assert e < 2e-5


def test_noalloc_refuses_requests_beyond_the_scratch(pnp):
    import torch
    n, L = 384, 32
    tr = synth.uneven_slice_traj(n, 16, True)
    plan = pnp.Plan(to_dev(tr.k), (n, n))
    tp = pnp.Toeplitz(plan)
    need = plan.workspace(L)[1]
    assert need > 64 << 20
    x = torch.zeros((n, n), dtype=torch.complex64, device="cuda")
    S = torch.zeros((L, n, n), dtype=torch.complex64, device="cuda")
    out = torch.full((n, n), 7.0, dtype=torch.complex64, device="cuda")
    with pytest.raises(pnp.PnPError) as ei:
        tp.normal_noalloc(x, S, out)
    assert ei.value.status == -5
    assert "static" in str(ei.value)
    assert bool((out == 7.0).all())          # nothing ran
