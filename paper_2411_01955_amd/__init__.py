"""MI355X-native multicoil non-Cartesian MRI operator and annealed PnP-HQS.

Python face of the C ABI in ``include/pnpmri.h`` (argument marshalling
only: every step runs in the HIP library).  PyTorch supplies device memory
and the current HIP stream.

    plan = Plan(traj, (ny, nx))          # traj: cuda float32 [M][2], radians
    y = plan.forward(x, smaps)           # A x,            [L][M] complex64
    x = plan.adjoint(y, smaps, dcf)      # A^H D_w y,      image complex64
    v = plan.normal(x, smaps, dcf)       # A^H D_w A x
    nrm = plan.opnorm(smaps, dcf)        # ||A^H D_w A||   (power iteration)
    x, rep = hqs_solve(plan, y, smaps, dcf, WaveletPrior(0, kappa), sigmas,
                       lam=..., precond="f1", n_cg=5)

    net = UNet(pack_unet_params(params))  # learned denoiser (BF16 MFMA kernels)
    d = net.forward(u, sigma)              # u + UNet([Re u, Im u, sigma])
    loss = net.backward(u, target)         # l1 loss, gradients into the net
    net.adam_step(1e-4)
    prior = UNetPrior(net, (ny, nx), kappa, fallback=WaveletPrior(0, kw))
"""
from __future__ import annotations

import ctypes as C
import os

from ._lib import HQSOpts, HQSReport, PnPError, PRECOND, UNET_BUF, Slice, Tuning, UNetLayer, check, load

__all__ = ["Plan", "Toeplitz", "WaveletPrior", "UNet", "UNetPrior", "hqs_solve", "PnPError", "load",
           "trace_enable", "trace_read", "unet_layers", "pack_unet_params", "unpack_unet_params",
           "UNET_LAYER_NAMES", "UNET_TENSORS", "trained_unet", "TRAINED_WEIGHTS", "Batch"]


def trace_enable(on: bool = True):
    """Start/stop bracketing every library kernel with HIP events."""
    check(load().pnp_trace_enable(1 if on else 0))


def trace_read():
    """{kernel: (launches, total_ms)} since the last read (waits for the events)."""
    import json
    buf = C.create_string_buffer(1 << 20)
    need = C.c_size_t()
    check(load().pnp_trace_read(buf, len(buf), C.byref(need)))
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _need_c64(t, name, shape=None):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex64):
        raise TypeError(f"{name} must be a CUDA complex64 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _need_f32(t, name, shape):
    torch = _torch()
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous CUDA float32 tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """Gridding plan for one trajectory (``traj``: CUDA float32 [M][d])."""

    def __init__(self, traj, shape):
        torch = _torch()
        lib = load()
        if not (isinstance(traj, torch.Tensor) and traj.is_cuda and traj.dtype == torch.float32):
            raise TypeError("traj must be a CUDA float32 tensor [M][d]")
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        if traj.dim() != 2 or traj.shape[1] != self.ndim:
            raise ValueError(f"traj must be [M][{self.ndim}]")
        self.traj = traj.contiguous()
        self.M = int(traj.shape[0])
        self.N = 1
        for s in self.shape:
            self.N *= s
        h = C.c_void_p()
        shp = (C.c_int32 * self.ndim)(*self.shape)
        check(lib.pnp_plan_create(C.byref(h), self.ndim, shp, self.M, _ptr(self.traj), _stream()))
        self._h = h
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        g = (C.c_int32 * self.ndim)()
        nt = C.c_int32()
        ne = C.c_int64()
        check(load().pnp_plan_info(self._h, g, C.byref(nt), C.byref(ne)))
        return {"grid": tuple(g), "tiles": nt.value, "entries": ne.value}

    def workspace(self, L, kind="op"):
        """Device workspace (cached per coil count and kind)."""
        torch = _torch()
        key = (kind, L)
        if key not in self._ws:
            n = C.c_size_t()
            fn = load().pnp_hqs_workspace_bytes if kind == "hqs" else load().pnp_workspace_bytes
            check(fn(self._h, L, C.byref(n)))
            self._ws[key] = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.traj.device)
        w = self._ws[key]
        return w, w.numel()

    def _L(self, smaps):
        _need_c64(smaps, "smaps")
        if tuple(smaps.shape[1:]) != self.shape:
            raise ValueError(f"smaps must be [L]{list(self.shape)}")
        return int(smaps.shape[0])

    def forward(self, x, smaps, out=None):
        L = self._L(smaps)
        _need_c64(x, "x", self.shape)
        y = out if out is not None else _torch().empty((L, self.M), dtype=_torch().complex64, device=x.device)
        _need_c64(y, "y", (L, self.M))
        ws, nb = self.workspace(L)
        check(load().pnp_forward(self._h, _ptr(x), _ptr(smaps), L, _ptr(y), _ptr(ws), nb, _stream()))
        return y

    def adjoint(self, y, smaps, dcf=None, out=None):
        L = self._L(smaps)
        _need_c64(y, "y", (L, self.M))
        _need_f32(dcf, "dcf", (self.M,))
        x = out if out is not None else _torch().empty(self.shape, dtype=_torch().complex64, device=y.device)
        _need_c64(x, "x", self.shape)
        ws, nb = self.workspace(L)
        check(load().pnp_adjoint(self._h, _ptr(y), _ptr(smaps), L, _ptr(dcf), _ptr(x), _ptr(ws), nb,
                                 _stream()))
        return x

    def normal(self, x, smaps, dcf=None, out=None):
        L = self._L(smaps)
        _need_c64(x, "x", self.shape)
        _need_f32(dcf, "dcf", (self.M,))
        o = out if out is not None else _torch().empty(self.shape, dtype=_torch().complex64, device=x.device)
        _need_c64(o, "out", self.shape)
        ws, nb = self.workspace(L)
        check(load().pnp_normal(self._h, _ptr(x), _ptr(smaps), L, _ptr(dcf), _ptr(o), _ptr(ws), nb,
                                _stream()))
        return o

    @property
    def row_coils(self):
        """Coils per workgroup of the register-FFT adjoint row pass (2, 4 or
        8; it also sets the coil groups of the partial images).  Assigning
        sets the forward and the adjoint pass."""
        v = C.c_int32()
        check(load().pnp_plan_get_row_coils(self._h, C.byref(v)))
        return v.value

    @row_coils.setter
    def row_coils(self, value):
        check(load().pnp_plan_set_row_coils(self._h, int(value)))

    @property
    def row_coils_pair(self):
        """(forward, adjoint) coils per workgroup of the row passes."""
        f, a = C.c_int32(), C.c_int32()
        check(load().pnp_plan_get_row_coils_pair(self._h, C.byref(f), C.byref(a)))
        return f.value, a.value

    @row_coils_pair.setter
    def row_coils_pair(self, value):
        f, a = value
        check(load().pnp_plan_set_row_coils_pair(self._h, int(f), int(a)))

    @property
    def spread(self):
        """(split level 0..3, dense-block threshold) of the 2D adjoint spread."""
        a, b = C.c_int32(), C.c_int32()
        check(load().pnp_plan_get_spread(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    @spread.setter
    def spread(self, value):
        split, dense_min = value
        check(load().pnp_plan_set_spread(self._h, int(split), int(dense_min), _stream()))

    def autotune(self, smaps, dcf=None, toeplitz=None, cache=None):
        """Time the normal operator for 2, 4 and 8 coils per row-pass
        workgroup, the adjoint pass first and then the forward one, and keep
        the fastest of each; `cache`: JSON-lines file (read and appended).
        Returns {row_coils (adjoint), row_coils_fwd, time_us (adjoint
        sweep), time_fwd_us (forward sweep), from_cache}."""
        L = self._L(smaps)
        _need_f32(dcf, "dcf", (self.M,))
        t = Tuning()
        t.struct_size = C.sizeof(Tuning)
        check(load().pnp_autotune(self._h, _ptr(smaps), L, _ptr(dcf),
                                  toeplitz.handle if toeplitz is not None else None,
                                  cache.encode() if cache else None, C.byref(t), _stream()))
        return {"row_coils": t.row_coils, "row_coils_fwd": t.row_coils_fwd, "time_us": list(t.time_us),
                "time_fwd_us": list(t.time_fwd_us), "from_cache": bool(t.from_cache),
                "spread_split": t.spread_split, "spread_dense_min": t.spread_dense_min,
                "time_spread_us": list(t.time_spread_us)}

    def opnorm(self, smaps, dcf=None, iters=50, seed=0):
        L = self._L(smaps)
        _need_f32(dcf, "dcf", (self.M,))
        ws, nb = self.workspace(L)
        v = C.c_double()
        check(load().pnp_opnorm(self._h, _ptr(smaps), L, _ptr(dcf), iters, seed, C.byref(v), _ptr(ws), nb,
                                _stream()))
        return v.value


class Toeplitz:
    """Toeplitz embedding of A^H D_w A for one plan and DCF (2D)."""

    def __init__(self, plan: Plan, dcf=None):
        _need_f32(dcf, "dcf", (plan.M,))
        self.plan = plan
        self._dcf = dcf
        h = C.c_void_p()
        check(load().pnp_toeplitz_create(C.byref(h), plan.handle, _ptr(dcf), _stream()))
        self._h = h

    @property
    def handle(self):
        return self._h

    def normal(self, x, smaps, out=None):
        L = self.plan._L(smaps)
        _need_c64(x, "x", self.plan.shape)
        o = out if out is not None else _torch().empty(self.plan.shape, dtype=_torch().complex64, device=x.device)
        _need_c64(o, "out", self.plan.shape)
        ws, nb = self.plan.workspace(L)
        check(load().pnp_normal_toeplitz(self._h, _ptr(x), _ptr(smaps), L, _ptr(o), _ptr(ws), nb, _stream()))
        return o

    def normal_noalloc(self, x, smaps, out):
        """The same operator through the entry point that allocates nothing
        (the library's static per-device scratch; ``out`` is required)."""
        L = self.plan._L(smaps)
        _need_c64(x, "x", self.plan.shape)
        _need_c64(out, "out", self.plan.shape)
        check(load().pnp_normal_toeplitz_noalloc(self._h, _ptr(x), _ptr(smaps), L, _ptr(out), _stream()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_toeplitz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WaveletPrior:
    """Haar soft-threshold prior, tau = kappa * sigma (levels 0: default rule)."""

    def __init__(self, levels: int = 0, kappa: float = 1.0):
        h = C.c_void_p()
        check(load().pnp_prior_wavelet(C.byref(h), int(levels), float(kappa)))
        self._h = h
        self.levels = levels
        self.kappa = kappa

    @property
    def handle(self):
        return self._h

    def __call__(self, u, sigma, out=None):
        _need_c64(u, "u")
        o = out if out is not None else _torch().empty_like(u)
        shp = (C.c_int32 * u.dim())(*u.shape)
        check(load().pnp_prior_apply(self._h, u.dim(), shp, _ptr(u), _ptr(o), float(sigma), _stream()))
        return o

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_prior_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hqs_solve(plan: Plan, y, smaps, dcf, prior, sigmas, lam: float, precond: str = "f1", n_cg: int = 5,
              opnorm: float = 0.0, opnorm_iters: int = 50, opnorm_seed: int = 0, x0=None,
              report: bool = False, out=None, rise_tol: float = 0.0, toeplitz: "Toeplitz" = None,
              k_start: int = 0):
    """Annealed preconditioned PnP-HQS; returns (x, report dict or None).
    With ``toeplitz`` the CG steps use the Toeplitz normal operator.  With
    ``k_start`` > 0 only iterations k_start.. of the schedule run, from
    ``x0`` (resume); the report lists those iterations."""
    torch = _torch()
    L = plan._L(smaps)
    _need_c64(y, "y", (L, plan.M))
    _need_f32(dcf, "dcf", (plan.M,))
    if x0 is not None:
        _need_c64(x0, "x0", plan.shape)
    n_out = len(sigmas)
    sig = (C.c_double * n_out)(*[float(s) for s in sigmas])
    if toeplitz is not None and toeplitz.plan is not plan:
        raise ValueError("toeplitz was built for another plan")
    o = HQSOpts(C.sizeof(HQSOpts), PRECOND[precond.lower()], int(n_cg), int(opnorm_iters), float(lam),
                float(opnorm), int(opnorm_seed), x0.data_ptr() if x0 is not None else None, float(rise_tol),
                toeplitz.handle.value if toeplitz is not None else None, int(k_start))
    x = out if out is not None else torch.empty(plan.shape, dtype=torch.complex64, device=y.device)
    _need_c64(x, "out", plan.shape)
    ws, nb = plan.workspace(L, "hqs")
    rep_p = None
    if report:
        rho = (C.c_double * n_out)()
        fb = (C.c_int32 * n_out)()
        rep = HQSReport(C.sizeof(HQSReport), n_out, rho, fb, 0.0)
        rep_p = C.byref(rep)
    check(load().pnp_hqs_solve(plan.handle, _ptr(y), _ptr(smaps), L, _ptr(dcf), prior.handle, sig, n_out,
                               C.byref(o), _ptr(x), rep_p, _ptr(ws), nb, _stream()))
    if report:
        return x, {"rho": list(rho)[k_start:], "fallback": list(fb)[k_start:], "opnorm": rep.opnorm_used}
    return x, None


def estimate_smaps(plan: Plan, y, dcf=None, width: float = 20.0, threshold: float = 0.05, out=None):
    """Coil sensitivity maps [L][shape] from the k-space centre of y [L][M]
    (Hamming window of `width` grid units, root-sum-of-squares, mask at
    `threshold` of the largest root sum of squares)."""
    torch = _torch()
    if not (isinstance(y, torch.Tensor) and y.dim() == 2):
        raise ValueError("y must be a [L][M] tensor")
    L = int(y.shape[0])
    _need_c64(y, "y", (L, plan.M))
    _need_f32(dcf, "dcf", (plan.M,))
    S = out if out is not None else torch.empty((L,) + tuple(plan.shape), dtype=torch.complex64, device=y.device)
    _need_c64(S, "out", (L,) + tuple(plan.shape))
    nb = C.c_size_t()
    check(load().pnp_smaps_workspace_bytes(plan.handle, C.byref(nb)))
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=y.device)
    check(load().pnp_smaps_estimate(plan.handle, _ptr(y), L, _ptr(dcf), float(width), float(threshold), _ptr(S),
                                    _ptr(ws), ws.numel(), _stream()))
    return S


def pgd_solve(plan: Plan, y, smaps, dcf, prior, sigmas, gamma: float, precond: str = "id", opnorm: float = 0.0,
              x0=None, out=None, toeplitz: "Toeplitz" = None):
    """PnP-PGD with one noise level per iteration (sigmas); returns x."""
    torch = _torch()
    L = plan._L(smaps)
    _need_c64(y, "y", (L, plan.M))
    _need_f32(dcf, "dcf", (plan.M,))
    if x0 is not None:
        _need_c64(x0, "x0", plan.shape)
    if toeplitz is not None and toeplitz.plan is not plan:
        raise ValueError("toeplitz was built for another plan")
    n = len(sigmas)
    sig = (C.c_double * n)(*[float(s) for s in sigmas])
    x = out if out is not None else torch.empty(plan.shape, dtype=torch.complex64, device=y.device)
    _need_c64(x, "out", plan.shape)
    ws, nb = plan.workspace(L, "hqs")
    check(load().pnp_pgd_solve(plan.handle, _ptr(y), _ptr(smaps), L, _ptr(dcf), prior.handle, sig, n, float(gamma),
                               PRECOND[precond.lower()], float(opnorm),
                               toeplitz.handle.value if toeplitz is not None else None,
                               x0.data_ptr() if x0 is not None else None, _ptr(x), _ptr(ws), nb, _stream()))
    return x


def fista_wavelet(plan: Plan, y, smaps, dcf, lam: float, gamma: float, n_iter: int, levels: int = 0, x0=None,
                  out=None, toeplitz: "Toeplitz" = None):
    """FISTA on f + lam ||detail(Haar x)||_1; returns x."""
    torch = _torch()
    L = plan._L(smaps)
    _need_c64(y, "y", (L, plan.M))
    _need_f32(dcf, "dcf", (plan.M,))
    if x0 is not None:
        _need_c64(x0, "x0", plan.shape)
    if toeplitz is not None and toeplitz.plan is not plan:
        raise ValueError("toeplitz was built for another plan")
    x = out if out is not None else torch.empty(plan.shape, dtype=torch.complex64, device=y.device)
    _need_c64(x, "out", plan.shape)
    ws, nb = plan.workspace(L, "hqs")
    check(load().pnp_fista_wavelet(plan.handle, _ptr(y), _ptr(smaps), L, _ptr(dcf), int(levels), float(lam),
                                   float(gamma), int(n_iter), toeplitz.handle.value if toeplitz is not None else None,
                                   x0.data_ptr() if x0 is not None else None, _ptr(x), _ptr(ws), nb, _stream()))
    return x


# ------------------------------------------------------------------ UNet
# Parameters trained by train_unet.py (2,000 seeded 320 x 320 phantoms, 100
# epochs, batch 10, 128 x 128 patches, sigma ~ U(0.001, 0.1), Adam 1e-4).
TRAINED_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_phantom.npz")


def trained_unet(path: str = TRAINED_WEIGHTS) -> "UNet":
    """The UNet with the packaged trained parameters."""
    import numpy as np
    with np.load(path, allow_pickle=False) as z:
        return UNet(z["params"].astype(np.float32))


UNET_LAYER_NAMES = ("e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "ba", "bb", "up3", "d3a", "d3b",
                    "up2", "d2a", "d2b", "up1", "d1a", "d1b", "out")
# workspace tensor ids of pnp_unet_tensor
UNET_TENSORS = ("x0", "e1a", "c1", "d1a", "d1b", "p1", "e2a", "c2", "d2a", "d2b", "p2", "e3a", "c3",
                "d3a", "d3b", "p3", "ba", "bb", "out",
                "gout", "gd1b", "gd1a", "gc1", "gd2b", "gd2a", "gc2", "gd3b", "gd3a", "gc3", "gbb", "gba",
                "gp3", "ge3a", "gp2", "ge2a", "gp1", "ge1a")


def unet_layers():
    """[{name, kind, cin, cin_padded, cout, taps, w_offset, b_offset}] of the library's network."""
    lib = load()
    out = []
    for i in range(lib.pnp_unet_layer_count()):
        li = UNetLayer()
        check(lib.pnp_unet_layer_info(i, C.byref(li)))
        out.append({"name": UNET_LAYER_NAMES[i], "kind": ("conv3", "conv1", "up")[li.kind], "cin": li.cin,
                    "cin_padded": li.cin_padded, "cout": li.cout, "taps": li.taps, "w_offset": li.w_offset,
                    "b_offset": li.b_offset})
    return out


def pack_unet_params(params):
    """{name: (W[cout][taps][cin], b[cout])} -> flat float32 numpy array in
    the library's layout (input channels zero-padded where it pads them)."""
    import numpy as np
    flat = np.zeros(int(load().pnp_unet_param_count()), dtype=np.float32)
    for l in unet_layers():
        W, b = params[l["name"]]
        W = np.asarray(W)
        if W.shape != (l["cout"], l["taps"], l["cin"]):
            raise ValueError(f"{l['name']}: weight shape {W.shape}, expected {(l['cout'], l['taps'], l['cin'])}")
        Wp = np.zeros((l["cout"], l["taps"], l["cin_padded"]), dtype=np.float32)
        Wp[:, :, :l["cin"]] = W
        flat[l["w_offset"]:l["w_offset"] + Wp.size] = Wp.ravel()
        flat[l["b_offset"]:l["b_offset"] + l["cout"]] = np.asarray(b, dtype=np.float32)
    return flat


def unpack_unet_params(flat):
    """Inverse of pack_unet_params (float64 arrays; padding dropped)."""
    import numpy as np
    flat = np.asarray(flat, dtype=np.float64)
    out = {}
    for l in unet_layers():
        n = l["cout"] * l["taps"] * l["cin_padded"]
        W = flat[l["w_offset"]:l["w_offset"] + n].reshape(l["cout"], l["taps"], l["cin_padded"])
        out[l["name"]] = (W[:, :, :l["cin"]].copy(), flat[l["b_offset"]:l["b_offset"] + l["cout"]].copy())
    return out


class UNet:
    """The learned denoiser on the current device (BF16 weights and
    activations, FP32 accumulation, FP32 master weights and Adam moments).
    ``params``: flat float32 parameters (numpy or CUDA tensor) in the
    library layout, or a {name: (W, b)} dict."""

    def __init__(self, params):
        torch = _torch()
        import numpy as np
        if isinstance(params, dict):
            params = pack_unet_params(params)
        if isinstance(params, np.ndarray):
            params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
        self.n_params = int(load().pnp_unet_param_count())
        if tuple(params.shape) != (self.n_params,) or params.dtype != torch.float32 or not params.is_cuda:
            raise ValueError(f"params must be CUDA float32 [{self.n_params}]")
        h = C.c_void_p()
        check(load().pnp_unet_create(C.byref(h), _ptr(params.contiguous()), _stream()))
        self._h = h
        self._ws = {}
        self._loss = torch.zeros(1, dtype=torch.float64, device="cuda")

    @property
    def handle(self):
        return self._h

    def workspace(self, B, H, W, train):
        torch = _torch()
        key = (B, H, W, bool(train))
        if key not in self._ws:
            n = C.c_size_t()
            check(load().pnp_unet_workspace_bytes(B, H, W, 1 if train else 0, C.byref(n)))
            self._ws[key] = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        w = self._ws[key]
        return w, w.numel()

    def _sigma(self, sigma, B):
        torch = _torch()
        if not isinstance(sigma, torch.Tensor):
            sigma = torch.full((B,), float(sigma), dtype=torch.float32, device="cuda") \
                if not hasattr(sigma, "__len__") else torch.tensor(sigma, dtype=torch.float32, device="cuda")
        _need_f32(sigma, "sigma", (B,))
        return sigma

    def forward(self, u, sigma, out=None, train=False):
        """u + UNet([Re u, Im u, sigma]) for u [B][H][W] (or [H][W]); sigma per image."""
        _need_c64(u, "u")
        u3 = u if u.dim() == 3 else u.reshape((1,) + tuple(u.shape))
        B, H, W = (int(s) for s in u3.shape)
        sig = self._sigma(sigma, B)
        o = out if out is not None else _torch().empty_like(u)
        _need_c64(o, "out", tuple(u.shape))
        ws, nb = self.workspace(B, H, W, train)
        check(load().pnp_unet_forward(self._h, _ptr(u3), _ptr(sig), B, H, W, _ptr(o), _ptr(ws), nb, _stream()))
        return o

    def backward(self, u, target):
        """l1 loss of the preceding ``forward(u, sigma, train=True)``; fills the
        gradients.  Returns the loss as a CUDA float64 tensor [1]."""
        _need_c64(u, "u")
        u3 = u if u.dim() == 3 else u.reshape((1,) + tuple(u.shape))
        _need_c64(target, "target", tuple(u.shape))
        B, H, W = (int(s) for s in u3.shape)
        ws, nb = self.workspace(B, H, W, True)
        check(load().pnp_unet_backward(self._h, _ptr(u3), _ptr(target), B, H, W, _ptr(self._loss), _ptr(ws), nb,
                                       _stream()))
        return self._loss

    def n2n_backward(self, x, codes, eta=2.0):
        """Neighbor2Neighbor loss of the noisy images x [B][H][W] with the pair
        codes [B][H/2][W/2] (uint8, 0..7); fills the gradients.  Returns the
        loss as a CUDA float64 tensor [1]."""
        torch = _torch()
        _need_c64(x, "x")
        x3 = x if x.dim() == 3 else x.reshape((1,) + tuple(x.shape))
        B, H, W = (int(s) for s in x3.shape)
        if not (isinstance(codes, torch.Tensor) and codes.is_cuda and codes.dtype == torch.uint8
                and codes.is_contiguous() and tuple(codes.shape) == (B, H // 2, W // 2)):
            raise TypeError("codes must be a contiguous CUDA uint8 tensor [B][H/2][W/2]")
        key = ("n2n", B, H, W)
        if key not in self._ws:
            n = C.c_size_t()
            check(load().pnp_n2n_workspace_bytes(B, H, W, C.byref(n)))
            self._ws[key] = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        ws = self._ws[key]
        check(load().pnp_n2n_backward(self._h, _ptr(x3), _ptr(codes), float(eta), B, H, W, _ptr(self._loss),
                                      _ptr(ws), ws.numel(), _stream()))
        return self._loss

    def adam_step(self, lr=1e-4, beta1=0.9, beta2=0.999, eps=1e-8):
        check(load().pnp_unet_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream()))

    def get(self, which="params"):
        t = _torch().empty(self.n_params, dtype=_torch().float32, device="cuda")
        check(load().pnp_unet_get(self._h, UNET_BUF[which], _ptr(t), _stream()))
        return t

    def set(self, which, values):
        torch = _torch()
        import numpy as np
        if isinstance(values, np.ndarray):
            values = torch.from_numpy(np.ascontiguousarray(values, dtype=np.float32)).cuda()
        _need_f32(values, which, (self.n_params,))
        check(load().pnp_unet_set(self._h, UNET_BUF[which], _ptr(values), _stream()))

    @property
    def step(self):
        v = C.c_int64()
        check(load().pnp_unet_get_step(self._h, C.byref(v)))
        return v.value

    @step.setter
    def step(self, value):
        check(load().pnp_unet_set_step(self._h, int(value)))

    def tensor(self, name, B, H, W, train):
        """View of a workspace activation as a CUDA tensor [B][h][w][C]
        (bfloat16; FP32 for 'out')."""
        torch = _torch()
        ws, _ = self.workspace(B, H, W, train)
        p = C.c_void_p()
        dims = (C.c_int32 * 4)()
        check(load().pnp_unet_tensor(B, H, W, 1 if train else 0, _ptr(ws), UNET_TENSORS.index(name), C.byref(p),
                                     dims))
        off = p.value - ws.data_ptr()
        n = dims[0] * dims[1] * dims[2] * dims[3]
        dt, es = (torch.float32, 4) if name == "out" else (torch.bfloat16, 2)
        return ws[off:off + n * es].view(dt).view(tuple(dims))

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UNetPrior:
    """Learned prior D_sigma(u) = UNet(u, kappa*sigma) for images of ``shape``,
    with an optional wavelet ``fallback`` used by hqs_solve where the
    data-consistency residual rises by more than ``rise_tol``."""

    def __init__(self, net: UNet, shape, kappa: float = 1.0, fallback: "WaveletPrior" = None):
        self.net, self.fallback = net, fallback
        self.shape = tuple(int(s) for s in shape)
        h = C.c_void_p()
        shp = (C.c_int32 * len(self.shape))(*self.shape)
        check(load().pnp_prior_unet(C.byref(h), net.handle, len(self.shape), shp, float(kappa),
                                    fallback.handle if fallback is not None else None))
        self._h = h

    @property
    def handle(self):
        return self._h

    def __call__(self, u, sigma, out=None):
        _need_c64(u, "u", self.shape)
        o = out if out is not None else _torch().empty_like(u)
        shp = (C.c_int32 * u.dim())(*u.shape)
        check(load().pnp_prior_apply(self._h, u.dim(), shp, _ptr(u), _ptr(o), float(sigma), _stream()))
        return o

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_prior_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- batches
class Batch:
    """Many 2D slices reconstructed together (one persistent launch per
    operator stage over all slices).  ``slices``: list of dicts with keys
    plan, toeplitz, y, smaps, dcf (or None), opnorm, lam and optionally out
    (the result tensor; allocated when absent)."""

    def __init__(self, slices):
        torch = _torch()
        self.slices = []
        arr = (Slice * len(slices))()
        for i, d in enumerate(slices):
            plan, tp = d["plan"], d["toeplitz"]
            L = plan._L(d["smaps"])
            _need_c64(d["y"], "y", (L, plan.M))
            _need_f32(d.get("dcf"), "dcf", (plan.M,))
            out = d.get("out")
            if out is None:
                out = torch.empty(plan.shape, dtype=torch.complex64, device=d["y"].device)
            _need_c64(out, "out", plan.shape)
            keep = dict(d, out=out, L=L)
            self.slices.append(keep)
            arr[i] = Slice(plan.handle.value, tp.handle.value, d["y"].data_ptr(), d["smaps"].data_ptr(), L,
                           d["dcf"].data_ptr() if d.get("dcf") is not None else None, float(d["opnorm"]),
                           float(d["lam"]), out.data_ptr())
        h = C.c_void_p()
        check(load().pnp_batch_create(C.byref(h), len(slices), arr, _stream()))
        self._h = h
        self._ws = {}

    @property
    def outputs(self):
        return [d["out"] for d in self.slices]

    def normal(self, xs, outs=None):
        """[A_i^H D_w A_i x_i] for every slice (Toeplitz operator)."""
        torch = _torch()
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for x, o, d in zip(xs, outs, self.slices):
            _need_c64(x, "x", d["plan"].shape)
            _need_c64(o, "out", d["plan"].shape)
        xa = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        oa = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        check(load().pnp_batch_normal(self._h, xa, oa, _stream()))
        return outs

    def hqs_solve(self, prior, sigmas, precond="f1", n_cg=5, report=False):
        """Annealed PnP-HQS of every slice; returns (outputs, rho [B][n_out] or None)."""
        torch = _torch()
        import numpy as np
        n_out = len(sigmas)
        sig = (C.c_double * n_out)(*[float(s) for s in sigmas])
        nb = C.c_size_t()
        check(load().pnp_batch_workspace_bytes(self._h, prior.handle, C.byref(nb)))
        key = nb.value
        if key not in self._ws:
            self._ws[key] = torch.empty(max(key, 256), dtype=torch.uint8, device="cuda")
        ws = self._ws[key]
        rho = (C.c_double * (len(self.slices) * n_out))() if report else None
        check(load().pnp_hqs_solve_batched(self._h, prior.handle, sig, n_out, PRECOND[precond.lower()], int(n_cg),
                                           rho, _ptr(ws), ws.numel(), _stream()))
        r = np.array(list(rho)).reshape(len(self.slices), n_out) if report else None
        return self.outputs, r

    def close(self):
        if getattr(self, "_h", None):
            load().pnp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
