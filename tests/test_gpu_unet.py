"""GPU parity of the UNet denoiser's BF16 MFMA kernels against the FP64
oracle (``oracle.unet``, BF16 rounding mirrored).

Per layer the oracle is fed the GPU's own BF16 inputs (teacher forcing), so
the comparison isolates one kernel: the only differences are FP32 vs FP64
accumulation, which flip an occasional BF16 rounding by one unit.  Bars:
per-layer forward and input gradients rel L2 <= 2e-3, weight gradients
<= 1e-3; the whole network (errors compounding over 18 layers) <= 1e-2 for
the output and 2e-2 for the gradients."""
import numpy as np
import pytest

import synth
from oracle import unet as U
from tests.gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pnp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_01955_amd as pnp
    pnp.load()
    return pnp


def _params(seed):
    p = synth.he_normal(U.param_shapes(), seed, last_scale={"out": 0.1})
    rng = np.random.default_rng(seed + 100)
    return {n: (W, rng.standard_normal(b.shape).astype(np.float32).astype(np.float64) * 0.02)
            for n, (W, b) in p.items()}


def _np(t):
    return t.float().cpu().numpy().astype(np.float64)


def _dev(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda() if dtype is None else \
        torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _setup(pnp, B, H, W, seed=3):
    params = _params(seed)
    net = pnp.UNet(params)
    u = (synth.white_complex((B, H, W), seed + 1) * 0.5).astype(np.complex64)
    sigma = np.linspace(0.05, 0.01, B).astype(np.float32)
    return params, net, u, sigma


def _acts(net, names, B, H, W, train=True):
    return {n: _np(net.tensor(n, B, H, W, train)) for n in names}


FWD = ("x0", "e1a", "c1", "d1a", "d1b", "p1", "e2a", "c2", "d2a", "d2b", "p2", "e3a", "c3", "d3a", "d3b",
       "p3", "ba", "bb", "out")


@pytest.mark.parametrize("B,H,W", [(2, 32, 40), (1, 40, 72)])
def test_forward_layers_teacher_forced(pnp, B, H, W):
    """(1, 40, 72): 8 x 16-pixel output patches cut at the right edge on every
    level (72 = 4.5 patches) and a 5 x 9 bottleneck; the max-pools and the
    output layer come from the convolutions' fused epilogues."""
    params, net, u, sigma = _setup(pnp, B, H, W)
    D = net.forward(_dev(u), _dev(sigma), train=True)
    a = _acts(net, FWD, B, H, W)
    R = U.bf16
    P = {n: (R(Wt), b) for n, (Wt, b) in params.items()}
    x0 = U.net_input(u, sigma)
    assert np.array_equal(a["x0"][..., :3], x0) and not a["x0"][..., 3:].any()

    def conv(name, x, act=True):
        z = U.conv(x, *P[name])
        return R(U.relu(z)) if act else z

    w1, w2, w3 = 32, 64, 128
    checks = [
        ("e1a", conv("e1a", a["x0"][..., :3]), a["e1a"]),
        ("e1b", conv("e1b", a["e1a"]), a["c1"][..., :w1]),
        ("p1", U.maxpool(a["c1"][..., :w1]), a["p1"]),
        ("e2a", conv("e2a", a["p1"]), a["e2a"]),
        ("e2b", conv("e2b", a["e2a"]), a["c2"][..., :w2]),
        ("p2", U.maxpool(a["c2"][..., :w2]), a["p2"]),
        ("e3a", conv("e3a", a["p2"]), a["e3a"]),
        ("e3b", conv("e3b", a["e3a"]), a["c3"][..., :w3]),
        ("p3", U.maxpool(a["c3"][..., :w3]), a["p3"]),
        ("ba", conv("ba", a["p3"]), a["ba"]),
        ("bb", conv("bb", a["ba"]), a["bb"]),
        ("up3", R(U.upconv(a["bb"], *P["up3"])), a["c3"][..., w3:]),
        ("d3a", conv("d3a", a["c3"]), a["d3a"]),
        ("d3b", conv("d3b", a["d3a"]), a["d3b"]),
        ("up2", R(U.upconv(a["d3b"], *P["up2"])), a["c2"][..., w2:]),
        ("d2a", conv("d2a", a["c2"]), a["d2a"]),
        ("d2b", conv("d2b", a["d2a"]), a["d2b"]),
        ("up1", R(U.upconv(a["d2b"], *P["up1"])), a["c1"][..., w1:]),
        ("d1a", conv("d1a", a["c1"]), a["d1a"]),
        ("d1b", conv("d1b", a["d1a"]), a["d1b"]),
        ("out", conv("out", a["d1b"], act=False), a["out"]),
    ]
    for name, ref, got in checks:
        e = rel_l2(got, ref)
        say(f"[unet fwd {B}x{H}x{W}] {name}: rel {e:.2e}  ({np.count_nonzero(got != ref)} of {ref.size} differ)")
        if name.startswith("p"):
            assert np.array_equal(got, ref), name     # max of identical BF16 values
        elif name == "out":
            assert e < 1e-5, name
        else:
            assert e < 2e-3, name
    out = a["out"]
    Dg = D.cpu().numpy()
    assert rel_l2(Dg, u + (out[..., 0] + 1j * out[..., 1])) < 1e-6


@pytest.mark.parametrize("B,H,W", [(2, 32, 32), (3, 48, 48), (1, 40, 72)])
def test_backward_layers_teacher_forced(pnp, B, H, W):
    """(3, 48, 48): the weight gradients of the full-resolution layers split
    over 11 pixel slices of 640 with a 512-pixel tail, and the 6 x 6
    bottleneck's 16-pixel steps wrap rows and images."""
    params, net, u, sigma = _setup(pnp, B, H, W, seed=5)
    target = (0.7 * u + 0.1 * synth.white_complex(u.shape, 6)).astype(np.complex64)
    ud, td = _dev(u), _dev(target)
    D = net.forward(ud, _dev(sigma), train=True)
    loss = float(net.backward(ud, td).item())
    a = _acts(net, FWD, B, H, W)
    gnames = ("gout", "gd1b", "gd1a", "gc1", "gd2b", "gd2a", "gc2", "gd3b", "gd3a", "gc3", "gbb", "gba", "gp3",
              "ge3a", "gp2", "ge2a", "gp1", "ge1a")
    g = _acts(net, gnames, B, H, W)
    grads = pnp.unpack_unet_params(net.get("grad").cpu().numpy())
    Dg = D.cpu().numpy().astype(np.complex128)
    assert abs(loss - U.l1_loss(Dg, target)) < 1e-6 * max(loss, 1e-12)
    R = U.bf16
    P = {n: (R(Wt), b) for n, (Wt, b) in params.items()}
    gout_ref = R(U.l1_grad(Dg, target))
    assert np.count_nonzero(g["gout"][..., :2] != gout_ref) <= 2 and not g["gout"][..., 2:].any()
    mask = lambda t: (t > 0).astype(np.float64)
    w1, w2, w3 = 32, 64, 128

    def split(c, w):
        m = np.ones_like(c)
        m[..., :w] = mask(c[..., :w])
        return m

    def cb(name, x, dz, m):
        dx, dW, db = U.conv_backward(x, P[name][0], dz)
        return (R(dx * m) if m is not None else R(dx)), dW, db

    def ub(name, x, dz, m):
        dx, dW, db = U.upconv_backward(x, P[name][0], dz)
        return R(dx * m), dW, db

    gouts = g["gout"][..., :2]
    steps = [
        # (layer, backward fn, layer input, dz (GPU), input-gradient mask, GPU input gradient)
        ("out", cb, a["d1b"], gouts, mask(a["d1b"]), g["gd1b"]),
        ("d1b", cb, a["d1a"], g["gd1b"], mask(a["d1a"]), g["gd1a"]),
        ("d1a", cb, a["c1"], g["gd1a"], split(a["c1"], w1), None),
        ("up1", ub, a["d2b"], g["gc1"][..., w1:], mask(a["d2b"]), g["gd2b"]),
        ("d2b", cb, a["d2a"], g["gd2b"], mask(a["d2a"]), g["gd2a"]),
        ("d2a", cb, a["c2"], g["gd2a"], split(a["c2"], w2), None),
        ("up2", ub, a["d3b"], g["gc2"][..., w2:], mask(a["d3b"]), g["gd3b"]),
        ("d3b", cb, a["d3a"], g["gd3b"], mask(a["d3a"]), g["gd3a"]),
        ("d3a", cb, a["c3"], g["gd3a"], split(a["c3"], w3), None),
        ("up3", ub, a["bb"], g["gc3"][..., w3:], mask(a["bb"]), g["gbb"]),
        ("bb", cb, a["ba"], g["gbb"], mask(a["ba"]), g["gba"]),
        ("ba", cb, a["p3"], g["gba"], None, g["gp3"]),
        ("e3b", cb, a["e3a"], g["gc3"][..., :w3], mask(a["e3a"]), g["ge3a"]),
        ("e3a", cb, a["p2"], g["ge3a"], None, g["gp2"]),
        ("e2b", cb, a["e2a"], g["gc2"][..., :w2], mask(a["e2a"]), g["ge2a"]),
        ("e2a", cb, a["p1"], g["ge2a"], None, g["gp1"]),
        ("e1b", cb, a["e1a"], g["gc1"][..., :w1], mask(a["e1a"]), g["ge1a"]),
        ("e1a", cb, a["x0"][..., :3], g["ge1a"], None, None),
    ]
    pre = {}
    for name, fn, x, dz, m, got in steps:
        dx, dW, db = fn(name, x, dz, m)
        eW, eb = rel_l2(grads[name][0], dW), rel_l2(grads[name][1], db)
        msg = f"[unet bwd {B}x{H}x{W}] {name}: dW {eW:.2e} db {eb:.2e}"
        if got is not None:
            ex = rel_l2(got, dx)
            msg += f" dX {ex:.2e}"
            assert ex < 2e-3, name
        else:
            pre[name] = dx
        say(msg)
        assert eW < 1e-3 and eb < 1e-3, name
    # skip gradients: decoder share (from the oracle's d*a input gradient)
    # plus the pooled share routed to the first maximum, masked, then rounded
    for dname, c, gc, gp, w in (("d1a", "c1", "gc1", "gp1", w1), ("d2a", "c2", "gc2", "gp2", w2),
                                ("d3a", "c3", "gc3", "gp3", w3)):
        skip = a[c][..., :w]
        ref = R(pre[dname][..., :w] + U.maxpool_backward(skip, g[gp]) * mask(skip))
        e = rel_l2(g[gc][..., :w], ref)
        eu = rel_l2(g[gc][..., w:], pre[dname][..., w:])
        say(f"[unet bwd] skip {gc}: rel {e:.2e}, up part {eu:.2e}")
        assert e < 2e-3 and eu < 2e-3


def test_whole_network_forward_backward(pnp):
    """No teacher forcing: both sides run the whole network from the same
    inputs.  The target sits 0.05 below the output in every component, so
    the l1 gradient has one sign everywhere and is the same on both sides.
    (With random signs every weight gradient is a cancelling sum, and the
    few ReLU-mask / max-pool decisions that one-ulp BF16 drift flips change
    it by several per cent: the oracle against itself with 20 input pixels
    moved by one BF16 ulp differs by 6% then, by 0.2% with one sign, and
    per layer by up to 5.5% in the 8x8 bottleneck, whose gradients sum over
    only 64 pixels.)  Per-layer kernel parity is the teacher-forced test's."""
    B, H, W = 1, 64, 64
    params, net, u, sigma = _setup(pnp, B, H, W, seed=7)
    D_ref, cache = U.forward(params, u, sigma)
    target = (D_ref - 0.05 * (1 + 1j)).astype(np.complex64)
    ud = _dev(u)
    D = net.forward(ud, _dev(sigma), train=True)
    net.backward(ud, _dev(target))
    grads = pnp.unpack_unet_params(net.get("grad").cpu().numpy())
    e = rel_l2(D.cpu().numpy() - u, D_ref - u)
    gout = U.l1_grad(D_ref, target)
    assert np.array_equal(np.sign(gout), np.sign(U.l1_grad(D.cpu().numpy().astype(np.complex128), target)))
    g_ref, _ = U.backward(params, cache, gout)
    errs = {n: max(rel_l2(grads[n][0], g_ref[n][0]), rel_l2(grads[n][1], g_ref[n][1])) for n in U.NAMES}
    flat = lambda G: np.concatenate([np.concatenate([G[n][0].ravel(), G[n][1].ravel()]) for n in U.NAMES])
    tot = rel_l2(flat(grads), flat(g_ref))
    say(f"[unet whole] output rel {e:.2e}, all gradients rel {tot:.2e}; per layer " +
        " ".join(f"{n}:{v:.1e}" for n, v in errs.items()))
    assert e < 1e-2
    assert tot < 1e-2
    assert max(errs.values()) < 6e-2


def test_whole_network_forward_128(pnp):
    """One 128 x 128 training-patch-sized image through the whole network."""
    B, H, W = 1, 128, 128
    params, net, u, sigma = _setup(pnp, B, H, W, seed=8)
    x, _ = synth.phantom2d(128, 8)
    u = (x + 0.03 * synth.white_complex(x.shape, 9))[None].astype(np.complex64)
    D = net.forward(_dev(u), _dev(sigma))
    D_ref, _ = U.forward(params, u, sigma)
    e = rel_l2(D.cpu().numpy() - u, D_ref - u)
    say(f"[unet whole] 128x128 output rel {e:.2e}")
    assert e < 1e-2


def test_whole_network_forward_large_tiles(pnp):
    """4 x 128 x 128 (65,536 pixels at full resolution, 16,384 at the second
    scale): the 32-channel full-resolution convolutions run on the 256 x 32
    tiles and the 64-channel second-scale ones on the 128 x 64 tiles."""
    B, H, W = 4, 128, 128
    params = _params(12)
    net = pnp.UNet(params)
    u = np.stack([(synth.phantom2d(128, 60 + i)[0] + 0.03 * synth.white_complex((H, W), 70 + i))
                  for i in range(B)]).astype(np.complex64)
    sigma = np.linspace(0.05, 0.01, B).astype(np.float32)
    D = net.forward(_dev(u), _dev(sigma))
    D_ref, _ = U.forward(params, u, sigma)
    e = rel_l2(D.cpu().numpy() - u, D_ref - u)
    say(f"[unet whole] 4x128x128 (large tiles) output rel {e:.2e}")
    assert e < 1e-2


def test_forward_batch_equals_single_images(pnp):
    """Six 320 x 320 images in one call give bit-identical outputs to six
    single-image calls.  The deep layers sum their K range in fixed chunks
    (2 or 4, set by the image size); a single image runs the chunks on
    parallel wave groups combined in order, the batch runs them in sequence
    on the 128 x 64 tiles, so the two must agree exactly."""
    B, H, W = 6, 320, 320
    params = _params(13)
    net = pnp.UNet(params)
    u = np.stack([(synth.phantom2d(H, 80 + i)[0] + 0.03 * synth.white_complex((H, W), 90 + i))
                  for i in range(B)]).astype(np.complex64)
    sigma = np.linspace(0.06, 0.01, B).astype(np.float32)
    Db = net.forward(_dev(u), _dev(sigma)).cpu().numpy()
    worst = 0.0
    for i in range(B):
        Di = net.forward(_dev(u[i:i + 1]), _dev(sigma[i:i + 1])).cpu().numpy()
        worst = max(worst, float(np.abs(Di[0] - Db[i]).max()))
    say(f"[unet batch] 6x320x320 vs single images: max |difference| {worst:.1e}")
    assert worst == 0.0


def test_adam_step_matches_oracle(pnp):
    B, H, W = 1, 16, 16
    params, net, u, sigma = _setup(pnp, B, H, W, seed=9)
    ud, td = _dev(u), _dev((0.5 * u).astype(np.complex64))
    opt = U.Adam(lr=1e-3)
    p_ref = pnp.unpack_unet_params(net.get("params").cpu().numpy())
    for it in range(3):
        net.forward(ud, _dev(sigma), train=True)
        net.backward(ud, td)
        g = pnp.unpack_unet_params(net.get("grad").cpu().numpy())
        net.adam_step(1e-3)
        p_ref = opt.step(p_ref, g)
        flat = net.get("params").cpu().numpy()
        got = pnp.unpack_unet_params(flat)
        worst = max(np.abs(got[n][j] - p_ref[n][j]).max() for n in U.NAMES for j in (0, 1))
        say(f"[unet adam] step {it + 1}: max |dw| {worst:.2e}")
        assert worst < 1e-6
    assert net.step == 3
    lay = pnp.unet_layers()[0]
    W0 = flat[:lay["cout"] * lay["taps"] * lay["cin_padded"]].reshape(lay["cout"], lay["taps"], -1)
    assert not W0[:, :, lay["cin"]:].any()        # the padding weights stay zero


def test_checkpoint_round_trip(pnp):
    """Parameters, Adam moments and the step count restore the training state."""
    B, H, W = 2, 16, 24
    params, net, u, sigma = _setup(pnp, B, H, W, seed=10)
    ud, sd, td = _dev(u), _dev(sigma), _dev((0.9 * u).astype(np.complex64))
    net.forward(ud, sd, train=True)
    net.backward(ud, td)
    net.adam_step(1e-3)
    net2 = pnp.UNet(net.get("params"))
    for which in ("adam_m", "adam_v"):
        net2.set(which, net.get(which))
    net2.step = net.step
    for n in (net, net2):
        n.forward(ud, sd, train=True)
        n.backward(ud, td)
        n.adam_step(1e-3)
    assert net2.step == net.step == 2
    a = net.forward(ud, sd).cpu().numpy()
    b = net2.forward(ud, sd).cpu().numpy()
    assert rel_l2(b - u, a - u) < 1e-4


def test_rejects_bad_shapes(pnp):
    import torch
    params, net, u, sigma = _setup(pnp, 1, 16, 16)
    x = torch.zeros((1, 20, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(pnp.PnPError) as ei:
        net.forward(x, _dev(sigma))
    assert ei.value.status == -2


def test_weight_gradients_are_deterministic(pnp):
    """Two backward passes over the same training batch (10 x 128 x 128, the
    training patch size) give bit-identical weight and bias gradients: each
    pixel slice's partial tile is added in a fixed order, no atomics."""
    B, H, W = 10, 128, 128
    params, net, u, sigma = _setup(pnp, B, H, W, seed=21)
    target = (0.8 * u).astype(np.complex64)
    ud, td, sd = _dev(u), _dev(target), _dev(sigma)
    runs = []
    for _ in range(2):
        net.forward(ud, sd, train=True)
        net.backward(ud, td)
        runs.append(pnp.unpack_unet_params(net.get("grad").cpu().numpy()))
    for n in U.NAMES:
        assert np.array_equal(runs[0][n][0], runs[1][n][0]) and np.array_equal(runs[0][n][1], runs[1][n][1]), n
        assert np.abs(runs[0][n][0]).max() > 0, n
    say(f"[unet bwd] {B}x{H}x{W}: all {len(U.NAMES)} layers' gradients bit-identical over two passes")


def test_training_reduces_the_loss(pnp):
    import torch
    B, H, W = 4, 64, 64
    params, net, _, _ = _setup(pnp, B, H, W, seed=12)
    clean = np.stack([synth.phantom2d(64, 20 + i)[0] for i in range(B)]).astype(np.complex64)
    noisy, sig = synth.denoise_pairs(clean, 0.02, 0.05, 13)
    nd, cd, sd = _dev(noisy), _dev(clean), _dev(sig)
    losses = []
    for it in range(80):
        net.forward(nd, sd, train=True)
        losses.append(float(net.backward(nd, cd).item()))
        net.adam_step(1e-3)
    torch.cuda.synchronize()
    say(f"[unet train] loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.7 * losses[0]


def test_new_network_starts_with_zero_adam_moments(pnp):
    """Moments of a network created where a trained one was freed are zero
    (every buffer is cleared on its own; the aligned blocks have gaps)."""
    import gc
    B, H, W = 1, 16, 16
    params, net, u, sigma = _setup(pnp, B, H, W, seed=10)
    ud = _dev(u)
    for _ in range(3):
        net.forward(ud, _dev(sigma), train=True)
        net.backward(ud, _dev((0.5 * u).astype(np.complex64)))
        net.adam_step(1e-3)
    net.close()
    del net
    gc.collect()
    fresh = pnp.UNet(params)
    for which in ("grad", "adam_m", "adam_v"):
        assert not fresh.get(which).cpu().numpy().any(), which
