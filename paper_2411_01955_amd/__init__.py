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
"""
from __future__ import annotations

import ctypes as C

from ._lib import HQSOpts, HQSReport, PnPError, PRECOND, check, load

__all__ = ["Plan", "Toeplitz", "WaveletPrior", "hqs_solve", "PnPError", "load", "trace_enable",
           "trace_read"]


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
              report: bool = False, out=None, rise_tol: float = 0.0, toeplitz: "Toeplitz" = None):
    """Annealed preconditioned PnP-HQS; returns (x, report dict or None).
    With ``toeplitz`` the CG steps use the Toeplitz normal operator."""
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
                toeplitz.handle.value if toeplitz is not None else None)
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
        return x, {"rho": list(rho), "fallback": list(fb), "opnorm": rep.opnorm_used}
    return x, None
