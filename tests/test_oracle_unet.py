"""Pins of the FP64 UNet oracle against libraries it does not use (torch's
CPU float64 convolutions, pooling, autograd and Adam; numpy's kron), central
finite differences, and hand-checked special cases."""
import math

import numpy as np
import pytest

import synth
from oracle import unet as U

torch = pytest.importorskip("torch")
F = torch.nn.functional

TINY = (4, 8, 16, 32)


def _t(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64)


def _conv_weight_torch(W):
    """W[o, t, c] -> torch weight [o, c, ky, kx] (t = 3 ky + kx)."""
    co, taps, ci = W.shape
    k = int(round(math.sqrt(taps)))
    return _t(W.reshape(co, k, k, ci).transpose(0, 3, 1, 2).copy())


def _up_weight_torch(W):
    """W[o, t, c] -> torch conv_transpose weight [c, o, a, b] (t = 2a + b)."""
    co, _, ci = W.shape
    return _t(W.reshape(co, 2, 2, ci).transpose(3, 0, 1, 2).copy())


def _nchw(x):
    return _t(np.ascontiguousarray(np.asarray(x).transpose(0, 3, 1, 2)))


def _nhwc(t):
    return t.detach().numpy().transpose(0, 2, 3, 1)


# ------------------------------------------------------------------ bf16
def test_bf16_matches_torch_bfloat16_rounding():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-40]])
    # exact halfway cases between two bf16 values: ties go to the even one
    base = np.array([1.0, 1.0078125, 3.0, -7.0], dtype=np.float32)
    half = (base.view(np.uint32) + 0x8000).view(np.float32).astype(np.float64)
    x = np.concatenate([x, half])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.bf16(x), ref)
    assert U.bf16(np.float64(1.0 + 2.0 ** -8)) == 1.0          # tie -> even (1.0)
    assert U.bf16(np.float64(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6   # tie -> even


# ------------------------------------------------------------- primitives
@pytest.mark.parametrize("taps", [9, 1])
def test_conv_matches_torch_conv2d(taps):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 7, 3))
    W = rng.standard_normal((4, taps, 3))
    b = rng.standard_normal(4)
    got = U.conv(x, W, b)
    ref = F.conv2d(_nchw(x), _conv_weight_torch(W), _t(b), padding=1 if taps == 9 else 0)
    np.testing.assert_allclose(got, _nhwc(ref), rtol=1e-12, atol=1e-12)


def test_conv_single_channel_matches_scipy_correlate():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(2)
    img = rng.standard_normal((6, 9))
    k = rng.standard_normal((3, 3))
    got = U.conv(img[None, :, :, None], k.reshape(1, 9, 1), np.zeros(1))[0, :, :, 0]
    np.testing.assert_allclose(got, correlate2d(img, k, mode="same", boundary="fill"), rtol=1e-12,
                               atol=1e-12)


def test_upconv_matches_torch_and_kron():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((6, 4, 5))
    b = rng.standard_normal(6)
    got = U.upconv(x, W, b)
    ref = F.conv_transpose2d(_nchw(x), _up_weight_torch(W), _t(b), stride=2)
    np.testing.assert_allclose(got, _nhwc(ref), rtol=1e-12, atol=1e-12)
    # one channel in and out: a Kronecker product with the 2x2 kernel
    k = rng.standard_normal((2, 2))
    img = rng.standard_normal((3, 4))
    one = U.upconv(img[None, :, :, None], k.reshape(1, 4, 1), np.zeros(1))[0, :, :, 0]
    np.testing.assert_allclose(one, np.kron(img, k), rtol=1e-12)


def test_maxpool_matches_torch_and_first_max_rule():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 8, 3))
    ref = F.max_pool2d(_nchw(x), 2)
    np.testing.assert_array_equal(U.maxpool(x), _nhwc(ref))
    # ties: the gradient goes to the first maximum in window order
    win = np.array([[1.0, 1.0], [1.0, 1.0]])[None, :, :, None]
    g = U.maxpool_backward(win, np.array([[[[5.0]]]]))
    assert g[0, 0, 0, 0] == 5.0 and g.sum() == 5.0
    win = np.array([[0.0, 2.0], [2.0, 0.0]])[None, :, :, None]
    g = U.maxpool_backward(win, np.array([[[[1.0]]]]))
    assert g[0, 0, 1, 0] == 1.0 and g.sum() == 1.0
    win = np.array([[-3.0, -1.0], [-2.0, -1.0]])[None, :, :, None]
    g = U.maxpool_backward(win, np.array([[[[2.0]]]]))
    assert g[0, 0, 1, 0] == 2.0 and g.sum() == 2.0


def test_primitive_gradients_match_torch_autograd():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 6, 4, 3))
    W = rng.standard_normal((5, 9, 3))
    dz = rng.standard_normal((2, 6, 4, 5))
    dx, dW, db = U.conv_backward(x, W, dz)
    xt = _nchw(x).requires_grad_()
    Wt = _conv_weight_torch(W).requires_grad_()
    bt = torch.zeros(5, dtype=torch.float64, requires_grad=True)
    (F.conv2d(xt, Wt, bt, padding=1) * _nchw(dz)).sum().backward()
    np.testing.assert_allclose(dx, _nhwc(xt.grad), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, Wt.grad.numpy().transpose(0, 2, 3, 1).reshape(5, 9, 3), rtol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11)
    # transposed convolution
    Wu = rng.standard_normal((4, 4, 3))
    du = rng.standard_normal((2, 12, 8, 4))
    dx, dW, db = U.upconv_backward(x, Wu, du)
    xt = _nchw(x).requires_grad_()
    Wt = _up_weight_torch(Wu).requires_grad_()
    bt = torch.zeros(4, dtype=torch.float64, requires_grad=True)
    (F.conv_transpose2d(xt, Wt, bt, stride=2) * _nchw(du)).sum().backward()
    np.testing.assert_allclose(dx, _nhwc(xt.grad), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dW, Wt.grad.numpy().transpose(1, 2, 3, 0).reshape(4, 4, 3), rtol=1e-11)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-11)
    # max-pool (no ties in random data)
    dp = rng.standard_normal((2, 3, 2, 3))
    xt = _nchw(x).requires_grad_()
    (F.max_pool2d(xt, 2) * _nchw(dp)).sum().backward()
    np.testing.assert_array_equal(U.maxpool_backward(x, dp), _nhwc(xt.grad))


# ------------------------------------------------------------- network
def _params(widths, seed, bias=0.0):
    """He-normal weights; with bias > 0, biases ~ N(0, bias^2) so that no
    preactivation sits exactly on a ReLU kink (dead inputs + zero bias)."""
    p = synth.he_normal(U.param_shapes(widths), seed)
    if bias:
        rng = np.random.default_rng(seed + 1)
        p = {n: (W, rng.standard_normal(b.shape) * bias) for n, (W, b) in p.items()}
    return p


def _torch_net(params, u, sigma):
    """The same network written with torch ops (float64, autograd)."""
    tp = {n: (_conv_weight_torch(W) if W.shape[1] in (1, 9) else _up_weight_torch(W), _t(b))
          for n, (W, b) in params.items()}
    for v in tp.values():
        v[0].requires_grad_()
        v[1].requires_grad_()
    x = _nchw(U.net_input(u, sigma, bf=False))

    def cv(n, z, act=True):
        W, b = tp[n]
        o = F.conv2d(z, W, b, padding=1 if W.shape[-1] == 3 else 0)
        return F.relu(o) if act else o

    def up(n, z):
        W, b = tp[n]
        return F.conv_transpose2d(z, W, b, stride=2)

    e1 = cv("e1b", cv("e1a", x))
    e2 = cv("e2b", cv("e2a", F.max_pool2d(e1, 2)))
    e3 = cv("e3b", cv("e3a", F.max_pool2d(e2, 2)))
    bb = cv("bb", cv("ba", F.max_pool2d(e3, 2)))
    d3 = cv("d3b", cv("d3a", torch.cat([e3, up("up3", bb)], 1)))
    d2 = cv("d2b", cv("d2a", torch.cat([e2, up("up2", d3)], 1)))
    d1 = cv("d1b", cv("d1a", torch.cat([e1, up("up1", d2)], 1)))
    return cv("out", d1, act=False), tp


def test_network_forward_and_gradients_match_torch_autograd():
    params = _params(TINY, 7)
    u = synth.white_complex((2, 16, 24), 8) * 0.5
    sigma = np.array([0.05, 0.01])
    D, cache = U.forward(params, u, sigma, bf16_mode=False, widths=TINY)
    out_t, tp = _torch_net(params, u, sigma)
    out = _nhwc(out_t)
    np.testing.assert_allclose(D - u, out[..., 0] + 1j * out[..., 1], rtol=1e-10, atol=1e-12)
    G = np.random.default_rng(9).standard_normal(out.shape)
    grads, _ = U.backward(params, cache, G, bf16_mode=False)
    (out_t * _nchw(G)).sum().backward()
    for n, (W, b) in params.items():
        Wg = tp[n][0].grad.numpy()
        if W.shape[1] == 4:
            Wg = Wg.transpose(1, 2, 3, 0).reshape(W.shape)
        else:
            Wg = Wg.transpose(0, 2, 3, 1).reshape(W.shape)
        np.testing.assert_allclose(grads[n][0], Wg, rtol=1e-9, atol=1e-12, err_msg=n)
        np.testing.assert_allclose(grads[n][1], tp[n][1].grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=n)


def test_network_gradients_by_central_differences():
    params = _params(TINY, 11, bias=0.1)
    u = synth.white_complex((1, 16, 16), 12) * 0.5
    sigma = np.array([0.03])
    G = np.random.default_rng(13).standard_normal((1, 16, 16, 2))

    def f(p):
        D, _ = U.forward(p, u, sigma, bf16_mode=False, widths=TINY)
        return float((G[..., 0] * (D - u).real).sum() + (G[..., 1] * (D - u).imag).sum())

    _, cache = U.forward(params, u, sigma, bf16_mode=False, widths=TINY)
    grads, _ = U.backward(params, cache, G, bf16_mode=False)
    rng = np.random.default_rng(14)
    h = 1e-6
    for n in U.NAMES:
        W, b = params[n]
        for j, arr in enumerate((W, b)):
            for _ in range(2):
                idx = tuple(int(rng.integers(s)) for s in arr.shape)
                pp = {k: (v[0].copy(), v[1].copy()) for k, v in params.items()}
                pm = {k: (v[0].copy(), v[1].copy()) for k, v in params.items()}
                pp[n][j][idx] += h
                pm[n][j][idx] -= h
                fd = (f(pp) - f(pm)) / (2 * h)
                an = grads[n][j][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (n, j, idx, fd, an)


def test_bf16_mode_rounds_every_stored_tensor_and_stays_close():
    params = _params(TINY, 15)
    u = synth.white_complex((1, 16, 16), 16) * 0.5
    D, a = U.forward(params, u, np.array([0.02]), bf16_mode=True, widths=TINY)
    D64, _ = U.forward(params, u, np.array([0.02]), bf16_mode=False, widths=TINY)
    for n in ("x0", "e1a", "c1", "p2", "bb", "d1b"):
        np.testing.assert_array_equal(U.bf16(a[n]), a[n])
    rel = np.linalg.norm(D - D64) / np.linalg.norm(D64 - u)
    assert rel < 5e-2
    G = U.l1_grad(D, u * 0.9)
    _, g = U.backward(params, a, G, bf16_mode=True)
    for n in ("gout", "gd1b", "gc1", "gs1", "ge1a"):
        np.testing.assert_array_equal(U.bf16(g[n]), g[n])


def test_param_count_of_the_full_network():
    # sum over layers of cout * taps * cin + cout
    assert U.param_count() == 1_925_634


# ------------------------------------------------------------- training
def test_l1_loss_and_gradient():
    D = np.array([[1 + 2j, 0.5 - 1j]])
    t = np.array([[1 + 1j, 1.0 - 1j]])
    assert U.l1_loss(D, t) == pytest.approx((0 + 1 + 0.5 + 0) / 4)
    g = U.l1_grad(D, t)
    np.testing.assert_array_equal(g[0, 0], [0.0, 0.25])     # sign(0) = 0
    np.testing.assert_array_equal(g[0, 1], [-0.25, 0.0])
    rng = np.random.default_rng(17)
    D = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    t = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    g = U.l1_grad(D, t)
    h = 1e-7
    for i in range(2):
        for j in range(3):
            e = np.zeros_like(D)
            e[i, j] = h
            assert (U.l1_loss(D + e, t) - U.l1_loss(D - e, t)) / (2 * h) == pytest.approx(g[i, j, 0], rel=1e-6)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(18)
    params = {"a": (rng.standard_normal((3, 4)), rng.standard_normal(3))}
    tw = [_t(params["a"][0]).requires_grad_(), _t(params["a"][1]).requires_grad_()]
    opt = torch.optim.Adam(tw, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    ad = U.Adam(lr=1e-3)
    for _ in range(4):
        g = (rng.standard_normal((3, 4)), rng.standard_normal(3))
        tw[0].grad, tw[1].grad = _t(g[0]), _t(g[1])
        opt.step()
        params = ad.step(params, {"a": g})
    np.testing.assert_allclose(params["a"][0], tw[0].detach().numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(params["a"][1], tw[1].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_is_lr_times_sign():
    ad = U.Adam(lr=0.01)
    p = {"a": (np.zeros(3), np.zeros(1))}
    out = ad.step(p, {"a": (np.array([2.0, -0.5, 0.0]), np.array([1e-3]))})
    np.testing.assert_allclose(out["a"][0], [-0.01, 0.01, 0.0], rtol=1e-7)
    np.testing.assert_allclose(out["a"][1], [-0.01], rtol=1e-4)


# ------------------------------------------------------- Neighbor2Neighbor
def test_n2n_subsample_hand_values():
    """4 x 4 image x[r, c] = 10 r + c, codes [[0, 3], [5, 6]]:
    cell (0,0) code 0 (0,0)->(0,1): 0, 1;   cell (0,1) code 3 (0,1)->(1,1): 3, 13;
    cell (1,0) code 5 (1,0)->(1,1): 30, 31; cell (1,1) code 6 (1,1)->(0,1): 33, 23."""
    x = (10 * np.arange(4)[:, None] + np.arange(4)[None, :]).astype(np.complex128)[None]
    g1, g2 = U.n2n_subsample(x, np.array([[[0, 3], [5, 6]]]))
    np.testing.assert_array_equal(g1[0].real, [[0, 3], [30, 33]])
    np.testing.assert_array_equal(g2[0].real, [[1, 13], [31, 23]])
    # every code is an ordered pair of distinct 4-adjacent pixels of the cell
    pairs = set()
    for a1, b1, a2, b2 in U.N2N_PAIRS:
        assert abs(a1 - a2) + abs(b1 - b2) == 1
        pairs.add((a1, b1, a2, b2))
    assert len(pairs) == 8


def test_n2n_identity_network_has_no_regulariser():
    """With a zero output layer f(u) = u, so e = g1(x) - g2(x) = d and the
    loss is the mean squared difference of the two sub-images, for any eta."""
    params = _params(TINY, 31)
    params["out"] = (np.zeros_like(params["out"][0]), np.zeros_like(params["out"][1]))
    x = synth.white_complex((2, 16, 16), 32).astype(np.complex128)
    codes = np.random.default_rng(33).integers(0, 8, (2, 8, 8))
    g1, g2 = U.n2n_subsample(x, codes)
    ref = float(np.mean(np.concatenate([(g1 - g2).real.ravel(), (g1 - g2).imag.ravel()]) ** 2))
    for eta in (0.0, 2.0):
        loss, _ = U.n2n_loss_grad(params, x, codes, eta, bf16_mode=False)
        assert abs(loss - ref) < 1e-12 * ref


def test_n2n_gradients_match_torch_autograd():
    """The same objective written with torch ops, f(x) detached."""
    params = _params(TINY, 34, bias=0.05)
    x = synth.white_complex((2, 16, 16), 35).astype(np.complex128) * 0.5
    codes = np.random.default_rng(36).integers(0, 8, (2, 8, 8))
    eta = 2.0
    loss, grads = U.n2n_loss_grad(params, x, codes, eta, bf16_mode=False)
    zeros = np.zeros(2)
    out_full, _ = _torch_net(params, x, zeros)
    f_full = _t(x.real) + out_full.detach()[:, 0], _t(x.imag) + out_full.detach()[:, 1]
    # sub-sampling written directly with the cell offsets of each code
    table = {0: ((0, 0), (0, 1)), 1: ((0, 0), (1, 0)), 2: ((0, 1), (0, 0)), 3: ((0, 1), (1, 1)),
             4: ((1, 0), (0, 0)), 5: ((1, 0), (1, 1)), 6: ((1, 1), (0, 1)), 7: ((1, 1), (1, 0))}
    B, h, w = codes.shape
    i1 = np.zeros((B, h, w, 2), dtype=int)
    i2 = np.zeros((B, h, w, 2), dtype=int)
    for b in range(B):
        for i in range(h):
            for j in range(w):
                (a1, c1), (a2, c2) = table[int(codes[b, i, j])]
                i1[b, i, j] = (2 * i + a1, 2 * j + c1)
                i2[b, i, j] = (2 * i + a2, 2 * j + c2)
    bb = np.arange(B)[:, None, None]
    sub = lambda a, ix: a[bb, ix[..., 0], ix[..., 1]]
    g1 = sub(x, i1)
    g2 = sub(x, i2)
    out_sub, tp = _torch_net(params, g1, zeros)
    D1r, D1i = _t(g1.real) + out_sub[:, 0], _t(g1.imag) + out_sub[:, 1]
    f1r, f1i = f_full[0][bb, i1[..., 0], i1[..., 1]], f_full[1][bb, i1[..., 0], i1[..., 1]]
    f2r, f2i = f_full[0][bb, i2[..., 0], i2[..., 1]], f_full[1][bb, i2[..., 0], i2[..., 1]]
    dr, di = D1r - _t(g2.real), D1i - _t(g2.imag)
    rr, ri = dr - (f1r - f2r), di - (f1i - f2i)
    L = (dr ** 2 + di ** 2 + eta * (rr ** 2 + ri ** 2)).sum() / (2 * dr.numel())
    L.backward()
    assert abs(L.item() - loss) < 1e-12 * loss
    for n, (W, b) in params.items():
        Wg = tp[n][0].grad.numpy()
        Wg = Wg.transpose(1, 2, 3, 0).reshape(W.shape) if W.shape[1] == 4 else Wg.transpose(0, 2, 3, 1).reshape(W.shape)
        np.testing.assert_allclose(grads[n][0], Wg, rtol=1e-9, atol=1e-13, err_msg=n)
        np.testing.assert_allclose(grads[n][1], tp[n][1].grad.numpy(), rtol=1e-9, atol=1e-13, err_msg=n)
