"""GPU parity of the coil sensitivity estimate from the k-space centre
against the FP64 oracle (``oracle.smaps``).

The maps are the low-resolution coil images over their root sum of squares
s, masked where s <= threshold * max s.  The mask is a floating-point
decision: pixels where the GPU and the oracle disagree must lie within a
relative 1e-4 of the threshold (the operator bar is 2e-5).  On the pixels
both keep, the maps agree within 4e-4 relative L2: the operator bar 2e-5
divided by the smallest kept s relative to its maximum (the threshold
0.05)."""
import numpy as np
import pytest

import synth
from oracle import ndft, smaps
from tests.gpu_util import rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu
THR = 0.05


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


@pytest.mark.parametrize("which", ["tiny", "clinical"])
def test_smaps_estimate_matches_oracle(pnp, which):
    w = synth.config_tiny() if which == "tiny" else synth.config_clinical()
    n, L = w.n, w.L
    k = w.traj.k
    M = k.shape[0]
    x, _ = synth.phantom2d(n, 21)
    S_true = synth.smaps2d(n, L)
    dcf = synth.voronoi_dcf(w.traj, n) if w.dcf else None
    y = (ndft.forward(x, S_true, k) + synth.complex_noise((L, M), synth.noise_variance(x, S_true), 22)).astype(
        np.complex64)
    S_ref, m_ref = smaps.estimate(y, k, (n, n), 20.0, dcf, THR)
    z = smaps.coil_images(y, k, (n, n), 20.0, dcf)
    s = np.sqrt((np.abs(z) ** 2).sum(0))
    plan = pnp.Plan(to_dev(k), (n, n))
    Sg = to_np(pnp.estimate_smaps(plan, to_dev(y), to_dev(dcf) if dcf is not None else None, 20.0, THR))
    m_gpu = np.any(Sg != 0, axis=0)
    flip = m_gpu != m_ref
    if flip.any():
        assert np.abs(s[flip] / s.max() - THR).max() < 1e-4
    assert flip.sum() <= max(2, 1e-3 * n * n)
    both = m_gpu & m_ref
    e = rel_l2(Sg[:, both], S_ref[:, both])
    sos = np.sqrt((np.abs(Sg[:, both]) ** 2).sum(0))
    say(f"[smaps] {which} n={n} L={L}: mask {m_ref.sum()} px, {flip.sum()} flipped, maps rel {e:.2e}, "
        f"SoS-1 {np.abs(sos - 1).max():.1e}")
    assert e < 4e-4
    assert np.abs(sos - 1).max() < 1e-5
    # inside the object the magnitudes are close to those of the maps that
    # made the data (the phases carry the object's own phase)
    roi = (np.abs(x) > 0) & both
    err_true = rel_l2(np.abs(Sg[:, roi]), np.abs(S_true[:, roi]))
    say(f"[smaps] {which}: magnitude distance to the true maps in the object {err_true:.3f}")
    assert err_true < 0.3


def test_smaps_rejects_bad_arguments(pnp):
    w = synth.config_tiny()
    plan = pnp.Plan(to_dev(w.traj.k), (w.n, w.n))
    y = to_dev(synth.white_complex((w.L, w.traj.k.shape[0]), 3))
    with pytest.raises(pnp.PnPError):
        pnp.estimate_smaps(plan, y, None, 0.0)
    with pytest.raises(pnp.PnPError):
        pnp.estimate_smaps(plan, y, None, 20.0, 1.5)
