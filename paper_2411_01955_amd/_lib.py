"""ctypes declarations of the C ABI in ``include/pnpmri.h``.

Loading fails loudly when ``libpnpmri.so`` has not been built: there is no
fallback implementation of any operation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpnpmri.so")

PNP_OK = 0
STATUS_NAMES = {0: "OK", -1: "ARG", -2: "SHAPE", -3: "UNSUPPORTED", -4: "DEVICE",
                -5: "WORKSPACE", -6: "NUMERIC"}

PRECOND = {"id": 0, "f1": 1, "cheb": 2}


class HQSOpts(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("precond", C.c_int32),
        ("n_cg", C.c_int32),
        ("opnorm_iters", C.c_int32),
        ("lam", C.c_double),
        ("opnorm", C.c_double),
        ("opnorm_seed", C.c_uint64),
        ("x0", C.c_void_p),
        ("rise_tol", C.c_double),
        ("toeplitz", C.c_void_p),
        ("k_start", C.c_int32),
    ]


class HQSReport(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("capacity", C.c_int32),
        ("rho", C.POINTER(C.c_double)),
        ("fallback", C.POINTER(C.c_int32)),
        ("opnorm_used", C.c_double),
    ]


class UNetLayer(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("cin", C.c_int32),
        ("cin_padded", C.c_int32),
        ("cout", C.c_int32),
        ("taps", C.c_int32),
        ("w_offset", C.c_int64),
        ("b_offset", C.c_int64),
    ]


UNET_BUF = {"params": 0, "grad": 1, "adam_m": 2, "adam_v": 3}


class Tuning(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("row_coils", C.c_int32),
        ("time_us", C.c_double * 3),
        ("from_cache", C.c_int32),
        ("row_coils_fwd", C.c_int32),
        ("time_fwd_us", C.c_double * 3),
        ("spread_split", C.c_int32),
        ("spread_dense_min", C.c_int32),
        ("time_spread_us", C.c_double * 12),
    ]


class Slice(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p),
        ("toeplitz", C.c_void_p),
        ("y", C.c_void_p),
        ("smaps", C.c_void_p),
        ("L", C.c_int32),
        ("dcf", C.c_void_p),
        ("opnorm", C.c_double),
        ("lam", C.c_double),
        ("x_out", C.c_void_p),
    ]

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_sz = C.c_size_t
_u64 = C.c_uint64
_dbl = C.c_double

# name: (restype, argtypes)
SIGNATURES = {
    "pnp_last_error": (C.c_char_p, []),
    "pnp_version": (_i32, []),
    "pnp_trace_enable": (_i32, [_i32]),
    "pnp_trace_read": (_i32, [C.c_char_p, _sz, C.POINTER(_sz)]),
    "pnp_plan_create": (_i32, [C.POINTER(_vp), _i32, C.POINTER(_i32), _i64, _vp, _vp]),
    "pnp_plan_destroy": (_i32, [_vp]),
    "pnp_plan_info": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i64)]),
    "pnp_workspace_bytes": (_i32, [_vp, _i32, C.POINTER(_sz)]),
    "pnp_forward": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "pnp_adjoint": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "pnp_normal": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _sz, _vp]),
    "pnp_opnorm": (_i32, [_vp, _vp, _i32, _vp, _i32, _u64, C.POINTER(_dbl), _vp, _sz, _vp]),
    "pnp_toeplitz_create": (_i32, [C.POINTER(_vp), _vp, _vp, _vp]),
    "pnp_toeplitz_destroy": (_i32, [_vp]),
    "pnp_normal_toeplitz": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]),
    "pnp_plan_set_spread": (_i32, [_vp, _i32, _i32, _vp]),
    "pnp_plan_get_spread": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    "pnp_noalloc_scratch_bytes": (_i32, [C.POINTER(_sz)]),
    "pnp_normal_toeplitz_noalloc": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "pnp_prior_wavelet": (_i32, [C.POINTER(_vp), _i32, _dbl]),
    "pnp_prior_destroy": (_i32, [_vp]),
    "pnp_prior_apply": (_i32, [_vp, _i32, C.POINTER(_i32), _vp, _vp, _dbl, _vp]),
    "pnp_hqs_workspace_bytes": (_i32, [_vp, _i32, C.POINTER(_sz)]),
    "pnp_hqs_solve": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, C.POINTER(_dbl), _i32,
                             C.POINTER(HQSOpts), _vp, C.POINTER(HQSReport), _vp, _sz, _vp]),
    "pnp_n2n_workspace_bytes": (_i32, [_i32, _i32, _i32, C.POINTER(_sz)]),
    "pnp_n2n_backward": (_i32, [_vp, _vp, _vp, _dbl, _i32, _i32, _i32, _vp, _vp, _sz, _vp]),
    "pnp_smaps_workspace_bytes": (_i32, [_vp, C.POINTER(_sz)]),
    "pnp_smaps_estimate": (_i32, [_vp, _vp, _i32, _vp, _dbl, _dbl, _vp, _vp, _sz, _vp]),
    "pnp_pgd_solve": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, C.POINTER(_dbl), _i32, _dbl, _i32, _dbl, _vp, _vp,
                             _vp, _vp, _sz, _vp]),
    "pnp_fista_wavelet": (_i32, [_vp, _vp, _vp, _i32, _vp, _i32, _dbl, _dbl, _i32, _vp, _vp, _vp, _vp, _sz,
                                 _vp]),
    "pnp_unet_layer_count": (_i32, []),
    "pnp_unet_param_count": (_i64, []),
    "pnp_unet_layer_info": (_i32, [_i32, C.POINTER(UNetLayer)]),
    "pnp_unet_create": (_i32, [C.POINTER(_vp), _vp, _vp]),
    "pnp_unet_destroy": (_i32, [_vp]),
    "pnp_unet_set": (_i32, [_vp, _i32, _vp, _vp]),
    "pnp_unet_get": (_i32, [_vp, _i32, _vp, _vp]),
    "pnp_unet_get_step": (_i32, [_vp, C.POINTER(_i64)]),
    "pnp_unet_set_step": (_i32, [_vp, _i64]),
    "pnp_unet_workspace_bytes": (_i32, [_i32, _i32, _i32, _i32, C.POINTER(_sz)]),
    "pnp_unet_forward": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp]),
    "pnp_unet_backward": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp]),
    "pnp_unet_adam_step": (_i32, [_vp, _dbl, _dbl, _dbl, _dbl, _vp]),
    "pnp_unet_tensor": (_i32, [_i32, _i32, _i32, _i32, _vp, _i32, C.POINTER(_vp), C.POINTER(_i32)]),
    "pnp_prior_unet": (_i32, [C.POINTER(_vp), _vp, _i32, C.POINTER(_i32), _dbl, _vp]),
    "pnp_autotune": (_i32, [_vp, _vp, _i32, _vp, _vp, C.c_char_p, C.POINTER(Tuning), _vp]),
    "pnp_plan_set_row_coils": (_i32, [_vp, _i32]),
    "pnp_plan_get_row_coils": (_i32, [_vp, C.POINTER(_i32)]),
    "pnp_plan_set_row_coils_pair": (_i32, [_vp, _i32, _i32]),
    "pnp_plan_get_row_coils_pair": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i32)]),
    "pnp_batch_create": (_i32, [C.POINTER(_vp), _i32, C.POINTER(Slice), _vp]),
    "pnp_batch_destroy": (_i32, [_vp]),
    "pnp_batch_normal": (_i32, [_vp, C.POINTER(_vp), C.POINTER(_vp), _vp]),
    "pnp_batch_workspace_bytes": (_i32, [_vp, _vp, C.POINTER(_sz)]),
    "pnp_hqs_solve_batched": (_i32, [_vp, _vp, C.POINTER(_dbl), _i32, _i32, _i32, C.POINTER(_dbl), _vp, _sz,
                                     _vp]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    # torch's HIP runtime must be the one in the process before the library
    # is mapped, so that both share a single runtime (same soname).
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2411_01955_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PnPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{STATUS_NAMES.get(status, status)}] {message}")
        self.status = status


def check(status: int):
    if status != PNP_OK:
        raise PnPError(status, load().pnp_last_error().decode(errors="replace"))
