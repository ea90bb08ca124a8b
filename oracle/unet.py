"""FP64 reference of the learned prior's UNet denoiser, its gradients, the
l1 training loss and Adam.  Test infrastructure: only the tests, the smoke
check and the benchmark's CPU baseline use it.

The denoiser (Sec. 2.3: complex images enter a real network as real and
imaginary channels; Sec. 4.2: noise-level conditioning, supervised l1 loss,
Adam) is read as a four-scale UNet:

  input   [Re u, Im u, sigma] (sigma as a constant map)
  encoder per scale two 3x3 convolutions ('same', zero padding) + ReLU,
          2x2 max-pool between scales
  decoder 2x2 stride-2 transposed convolution, concatenation [skip, up],
          two 3x3 convolutions + ReLU
  output  1x1 convolution to two channels;  D(u) = u + output

Every function is the plain definition of its operation: convolution as
cross-correlation written through im2col and a matrix product, its input
gradient as the adjoint (col2im) of that, pooling as a maximum over the
window with the first maximum (window order (0,0), (0,1), (1,0), (1,1))
taking the gradient.

With ``bf16=True`` values are rounded to bfloat16 (round to nearest even,
through float32) at the points where the GPU path stores BF16: the network
input, every stored activation, every stored activation gradient and the
loss gradient.  Sums stay in FP64.  With ``bf16=False`` the whole network is
FP64 (used for the finite-difference and library pins).

Layouts: activations [B, H, W, C]; conv weights W[cout, taps, cin] with
tap = 3*(dy+1) + (dx+1); transposed-conv weights W[cout, 4, cin] with
tap = 2a + b for output pixel (2i+a, 2j+b).
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128, 256)

# layer kinds
CONV3, CONV1, UP = "conv3", "conv1", "up"

# names in forward order
NAMES = ("e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "ba", "bb",
         "up3", "d3a", "d3b", "up2", "d2a", "d2b", "up1", "d1a", "d1b", "out")


def architecture(widths=WIDTHS):
    """[(name, kind, cin, cout)] of the four-scale UNet with the given widths."""
    w1, w2, w3, w4 = widths
    return [("e1a", CONV3, 3, w1), ("e1b", CONV3, w1, w1),
            ("e2a", CONV3, w1, w2), ("e2b", CONV3, w2, w2),
            ("e3a", CONV3, w2, w3), ("e3b", CONV3, w3, w3),
            ("ba", CONV3, w3, w4), ("bb", CONV3, w4, w4),
            ("up3", UP, w4, w3), ("d3a", CONV3, 2 * w3, w3), ("d3b", CONV3, w3, w3),
            ("up2", UP, w3, w2), ("d2a", CONV3, 2 * w2, w2), ("d2b", CONV3, w2, w2),
            ("up1", UP, w2, w1), ("d1a", CONV3, 2 * w1, w1), ("d1b", CONV3, w1, w1),
            ("out", CONV1, w1, 2)]


def taps_of(kind):
    return {CONV3: 9, CONV1: 1, UP: 4}[kind]


def param_shapes(widths=WIDTHS):
    """{name: (weight shape, bias shape)}"""
    return {n: ((co, taps_of(k), ci), (co,)) for n, k, ci, co in architecture(widths)}


def param_count(widths=WIDTHS):
    return sum(int(np.prod(w)) + b[0] for w, b in param_shapes(widths).values())


# ------------------------------------------------------------------ bf16
def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _rnd(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


# ------------------------------------------------------------- primitives
_OFFS = [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def im2col(x, taps):
    """cols[B, H, W, taps, C]: x at pixel + offset(tap), zero outside."""
    if taps == 1:
        return x[:, :, :, None, :]
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:H + 1, 1:W + 1] = x
    cols = np.empty((B, H, W, 9, C))
    for t, (dy, dx) in enumerate(_OFFS):
        cols[:, :, :, t, :] = xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
    return cols


def col2im(dcols, taps):
    """Adjoint of im2col: dx[pixel + offset(tap)] += dcols[pixel, tap]."""
    if taps == 1:
        return dcols[:, :, :, 0, :].copy()
    B, H, W, _, C = dcols.shape
    dxp = np.zeros((B, H + 2, W + 2, C))
    for t, (dy, dx) in enumerate(_OFFS):
        dxp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] += dcols[:, :, :, t, :]
    return dxp[:, 1:H + 1, 1:W + 1, :]


def conv(x, W, b):
    """out[p, o] = b[o] + sum_{t, c} x[p + off(t), c] W[o, t, c]."""
    B, H, Wd, C = x.shape
    co, taps, ci = W.shape
    assert ci == C
    cols = im2col(x, taps).reshape(-1, taps * C)
    return (cols @ W.reshape(co, -1).T + b).reshape(B, H, Wd, co)


def conv_backward(x, W, dz):
    """Gradients of conv for output gradient dz: (dx, dW, db)."""
    B, H, Wd, C = x.shape
    co, taps, ci = W.shape
    dzf = dz.reshape(-1, co)
    cols = im2col(x, taps).reshape(-1, taps * C)
    dW = (dzf.T @ cols).reshape(co, taps, ci)
    db = dzf.sum(0)
    dx = col2im((dzf @ W.reshape(co, -1)).reshape(B, H, Wd, taps, C), taps)
    return dx, dW, db


def upconv(x, W, b):
    """out[2i+a, 2j+b', o] = b[o] + sum_c x[i, j, c] W[o, 2a+b', c]."""
    B, h, w, C = x.shape
    co = W.shape[0]
    out = np.empty((B, 2 * h, 2 * w, co))
    for t in range(4):
        a, bb = divmod(t, 2)
        out[:, a::2, bb::2, :] = x @ W[:, t, :].T + b
    return out


def upconv_backward(x, W, dout):
    B, h, w, C = x.shape
    co = W.shape[0]
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t in range(4):
        a, bb = divmod(t, 2)
        g = dout[:, a::2, bb::2, :]
        dx += g @ W[:, t, :]
        dW[:, t, :] = g.reshape(-1, co).T @ x.reshape(-1, C)
    return dx, dW, dout.reshape(-1, co).sum(0)


def _windows(x):
    """[B, H/2, W/2, C, 4] in window order (0,0), (0,1), (1,0), (1,1)."""
    return np.stack([x[:, 0::2, 0::2], x[:, 0::2, 1::2], x[:, 1::2, 0::2], x[:, 1::2, 1::2]], axis=-1)


def maxpool(x):
    return _windows(x).max(axis=-1)


def maxpool_backward(x, dp):
    """Gradient routed to the first maximum of each window."""
    arg = _windows(x).argmax(axis=-1)   # first occurrence of the maximum
    dx = np.zeros_like(x)
    for q, (a, b) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        dx[:, a::2, b::2] = np.where(arg == q, dp, 0.0)
    return dx


def relu(z):
    return np.maximum(z, 0.0)


# ------------------------------------------------------------ the network
def net_input(u, sigma, bf=True):
    """[B, H, W, 3] = (Re u, Im u, sigma_b); u complex [B, H, W], sigma [B]."""
    u = np.asarray(u)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64).reshape(-1, 1, 1), u.shape)
    return _rnd(np.stack([u.real, u.imag, sig], axis=-1), bf)


def forward(params, u, sigma, bf16_mode=True, widths=WIDTHS):
    """Returns (D(u) complex [B, H, W], cache).  params: {name: (W, b)}."""
    arch = {n: (k, ci, co) for n, k, ci, co in architecture(widths)}
    R = lambda v: _rnd(v, bf16_mode)
    a = {"x0": net_input(u, sigma, bf16_mode)}

    def cv(name, x, act=True):
        W, b = params[name]
        z = conv(x, R(W), b)
        return R(relu(z)) if act else z

    def up(name, x):
        W, b = params[name]
        return R(upconv(x, R(W), b))

    a["e1a"] = cv("e1a", a["x0"])
    a["e1b"] = cv("e1b", a["e1a"])
    a["p1"] = maxpool(a["e1b"])
    a["e2a"] = cv("e2a", a["p1"])
    a["e2b"] = cv("e2b", a["e2a"])
    a["p2"] = maxpool(a["e2b"])
    a["e3a"] = cv("e3a", a["p2"])
    a["e3b"] = cv("e3b", a["e3a"])
    a["p3"] = maxpool(a["e3b"])
    a["ba"] = cv("ba", a["p3"])
    a["bb"] = cv("bb", a["ba"])
    a["up3"] = up("up3", a["bb"])
    a["c3"] = np.concatenate([a["e3b"], a["up3"]], axis=-1)
    a["d3a"] = cv("d3a", a["c3"])
    a["d3b"] = cv("d3b", a["d3a"])
    a["up2"] = up("up2", a["d3b"])
    a["c2"] = np.concatenate([a["e2b"], a["up2"]], axis=-1)
    a["d2a"] = cv("d2a", a["c2"])
    a["d2b"] = cv("d2b", a["d2a"])
    a["up1"] = up("up1", a["d2b"])
    a["c1"] = np.concatenate([a["e1b"], a["up1"]], axis=-1)
    a["d1a"] = cv("d1a", a["c1"])
    a["d1b"] = cv("d1b", a["d1a"])
    a["out"] = cv("out", a["d1b"], act=False)           # FP64 / FP32 output, not rounded
    D = np.asarray(u) + (a["out"][..., 0] + 1j * a["out"][..., 1])
    assert set(arch) == set(NAMES)
    return D, a


def backward(params, a, gout, bf16_mode=True):
    """Gradients {name: (dW, db)} for the output gradient gout [B, H, W, 2]
    (d loss / d output), and the activation gradients (dict)."""
    R = lambda v: _rnd(v, bf16_mode)
    P = {n: (R(W), b) for n, (W, b) in params.items()}
    g = {}
    grads = {}
    mask = lambda act: (act > 0).astype(np.float64)

    def cvb(name, x, dz, in_mask):
        """dz: gradient at the conv output (mask already applied)."""
        dx, dW, db = conv_backward(x, P[name][0], dz)
        grads[name] = (dW, db)
        return R(dx * in_mask) if in_mask is not None else R(dx)

    def upb(name, x, dz, in_mask):
        dx, dW, db = upconv_backward(x, P[name][0], dz)
        grads[name] = (dW, db)
        return R(dx * in_mask)

    def split_mask(c, skip):
        m = np.ones_like(c)
        m[..., :skip.shape[-1]] = mask(skip)
        return m

    g["gout"] = R(gout)
    g["gd1b"] = cvb("out", a["d1b"], g["gout"], mask(a["d1b"]))
    g["gd1a"] = cvb("d1b", a["d1a"], g["gd1b"], mask(a["d1a"]))
    g["gc1"] = cvb("d1a", a["c1"], g["gd1a"], split_mask(a["c1"], a["e1b"]))
    w1 = a["e1b"].shape[-1]
    g["gd2b"] = upb("up1", a["d2b"], g["gc1"][..., w1:], mask(a["d2b"]))
    g["gd2a"] = cvb("d2b", a["d2a"], g["gd2b"], mask(a["d2a"]))
    g["gc2"] = cvb("d2a", a["c2"], g["gd2a"], split_mask(a["c2"], a["e2b"]))
    w2 = a["e2b"].shape[-1]
    g["gd3b"] = upb("up2", a["d3b"], g["gc2"][..., w2:], mask(a["d3b"]))
    g["gd3a"] = cvb("d3b", a["d3a"], g["gd3b"], mask(a["d3a"]))
    g["gc3"] = cvb("d3a", a["c3"], g["gd3a"], split_mask(a["c3"], a["e3b"]))
    w3 = a["e3b"].shape[-1]
    g["gbb"] = upb("up3", a["bb"], g["gc3"][..., w3:], mask(a["bb"]))
    g["gba"] = cvb("bb", a["ba"], g["gbb"], mask(a["ba"]))
    g["gp3"] = cvb("ba", a["p3"], g["gba"], None)
    # skip gradients: decoder share (already masked) + pooled share, masked
    gs3 = R(g["gc3"][..., :w3] + maxpool_backward(a["e3b"], g["gp3"]) * mask(a["e3b"]))
    g["ge3a"] = cvb("e3b", a["e3a"], gs3, mask(a["e3a"]))
    g["gp2"] = cvb("e3a", a["p2"], g["ge3a"], None)
    gs2 = R(g["gc2"][..., :w2] + maxpool_backward(a["e2b"], g["gp2"]) * mask(a["e2b"]))
    g["ge2a"] = cvb("e2b", a["e2a"], gs2, mask(a["e2a"]))
    g["gp1"] = cvb("e2a", a["p1"], g["ge2a"], None)
    gs1 = R(g["gc1"][..., :w1] + maxpool_backward(a["e1b"], g["gp1"]) * mask(a["e1b"]))
    g["ge1a"] = cvb("e1b", a["e1a"], gs1, mask(a["e1a"]))
    dx0, dW, db = conv_backward(a["x0"], P["e1a"][0], g["ge1a"])
    grads["e1a"] = (dW, db)
    g["gs1"], g["gs2"], g["gs3"] = gs1, gs2, gs3
    return grads, g


# ------------------------------------------------------------- training
def l1_loss(D, target):
    """mean over the 2BHW real values of |D - target|."""
    d = np.asarray(D) - np.asarray(target)
    return float(np.mean(np.concatenate([np.abs(d.real).ravel(), np.abs(d.imag).ravel()])))


def l1_grad(D, target):
    """d l1 / d output [B, H, W, 2]: sign(D - target)/(2BHW), sign(0) = 0."""
    d = np.asarray(D) - np.asarray(target)
    n = 2 * d.size
    return np.stack([np.sign(d.real), np.sign(d.imag)], axis=-1) / n


class Adam:
    """Adam with bias-corrected moments (Kingma & Ba, Algorithm 1):
    m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""

    def __init__(self, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = {}
        self.v = {}

    def step(self, params, grads):
        self.t += 1
        out = {}
        for n, (W, b) in params.items():
            new = []
            for j, (w, gw) in enumerate(zip((W, b), grads[n])):
                key = (n, j)
                m = self.b1 * self.m.get(key, 0.0) + (1 - self.b1) * gw
                v = self.b2 * self.v.get(key, 0.0) + (1 - self.b2) * gw * gw
                self.m[key], self.v[key] = m, v
                mh = m / (1 - self.b1 ** self.t)
                vh = v / (1 - self.b2 ** self.t)
                new.append(w - self.lr * mh / (np.sqrt(vh) + self.eps))
            out[n] = tuple(new)
        return out


# ------------------------------------------------- Neighbor2Neighbor (Sec. 3.1)
# Ordered pairs of 4-adjacent pixels of a 2 x 2 cell, (dy1, dx1, dy2, dx2):
# the first goes to the sub-image g1, the second to g2.
N2N_PAIRS = ((0, 0, 0, 1), (0, 0, 1, 0), (0, 1, 0, 0), (0, 1, 1, 1),
             (1, 0, 0, 0), (1, 0, 1, 1), (1, 1, 0, 1), (1, 1, 1, 0))


def n2n_subsample(x, codes):
    """(g1, g2) [B, H/2, W/2]: in cell (i, j) of image b, pair N2N_PAIRS[codes[b, i, j]]."""
    x = np.asarray(x)
    codes = np.asarray(codes)
    B, h, w = codes.shape
    pairs = np.asarray(N2N_PAIRS)[codes]            # [B, h, w, 4]
    bi = np.arange(B)[:, None, None]
    ii = 2 * np.arange(h)[None, :, None]
    jj = 2 * np.arange(w)[None, None, :]
    g1 = x[bi, ii + pairs[..., 0], jj + pairs[..., 1]]
    g2 = x[bi, ii + pairs[..., 2], jj + pairs[..., 3]]
    return g1, g2


def n2n_loss(D1, g2, f1, f2, eta: float):
    """mean over the 2P real values of |d|^2 + eta |d - e|^2 (per real
    component), d = D1 - g2 = f(g1(x)) - g2(x), e = f1 - f2 = g1(f(x)) - g2(f(x))."""
    d = np.asarray(D1) - np.asarray(g2)
    r = d - (np.asarray(f1) - np.asarray(f2))
    n = 2 * d.size
    return float((np.sum(np.abs(d) ** 2) + eta * np.sum(np.abs(r) ** 2)) / n)


def n2n_loss_grad(params, x, codes, eta: float, bf16_mode=True):
    """Loss and parameter gradients of the Neighbor2Neighbor objective for the
    network without noise conditioning (sigma input 0), f(x) held constant:
    d loss / d f(g1(x)) = 2 (d + eta (d - e)) / (2P)."""
    x = np.asarray(x, dtype=np.complex128)
    B = x.shape[0]
    zeros = np.zeros(B)
    Dx, _ = forward(params, x, zeros, bf16_mode)
    g1, g2 = n2n_subsample(x, codes)
    f1, f2 = n2n_subsample(Dx, codes)
    D1, a = forward(params, g1, zeros, bf16_mode)
    loss = n2n_loss(D1, g2, f1, f2, eta)
    d = D1 - g2
    r = d - (f1 - f2)
    gc = 2.0 * (d + eta * r) / (2 * d.size)
    gout = np.stack([gc.real, gc.imag], axis=-1)
    grads, _ = backward(params, a, gout, bf16_mode)
    return loss, grads
