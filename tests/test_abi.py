"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point the header declares, and rejects invalid arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnpmri.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pnp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2411_01955_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpnpmri.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_and_binding_agree(lib):
    from paper_2411_01955_amd import _lib
    names = _declared()
    assert len(names) >= 14
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.pnp_version() >= 100


def test_null_arguments_rejected(lib):
    from paper_2411_01955_amd._lib import PNP_OK
    h = C.c_void_p()
    shape = (C.c_int32 * 2)(64, 64)
    assert lib.pnp_plan_create(None, 2, shape, 10, C.c_void_p(1), None) == -1
    assert b"out" in lib.pnp_last_error()
    assert lib.pnp_plan_create(C.byref(h), 2, None, 10, C.c_void_p(1), None) == -1
    assert lib.pnp_plan_create(C.byref(h), 2, shape, 10, None, None) == -1
    n = C.c_size_t()
    assert lib.pnp_workspace_bytes(None, 4, C.byref(n)) == -1
    assert lib.pnp_forward(None, None, None, 4, None, None, 0, None) == -1
    assert lib.pnp_hqs_solve(None, None, None, 1, None, None, None, 1, None, None, None, None, 0, None) == -1
    assert lib.pnp_plan_destroy(None) == PNP_OK


def test_plan_shape_validation_before_device_work(lib):
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)   # never dereferenced: shape checks come first
    bad_shapes = [(2, (C.c_int32 * 2)(63, 64)),      # odd
                  (2, (C.c_int32 * 2)(2, 64)),       # too small
                  (2, (C.c_int32 * 2)(64, 2048)),    # too large
                  (2, (C.c_int32 * 2)(64, 14)),      # 28 has factor 7
                  (4, (C.c_int32 * 4)(8, 8, 8, 8))]  # ndim
    for nd, shp in bad_shapes:
        assert lib.pnp_plan_create(C.byref(h), nd, shp, 16, fake, None) == -2, lib.pnp_last_error()
    assert lib.pnp_plan_create(C.byref(h), 2, (C.c_int32 * 2)(64, 64), 0, fake, None) == -2


def test_prior_validation_and_lifecycle(lib):
    h = C.c_void_p()
    assert lib.pnp_prior_wavelet(C.byref(h), -1, 1.0) == -1
    assert lib.pnp_prior_wavelet(C.byref(h), 2, float("nan")) == -1
    assert lib.pnp_prior_wavelet(C.byref(h), 0, 1.5) == 0
    shp = (C.c_int32 * 2)(64, 64)
    assert lib.pnp_prior_apply(h, 2, shp, None, None, 0.1, None) == -1
    assert lib.pnp_prior_apply(h, 5, shp, C.c_void_p(1), C.c_void_p(1), 0.1, None) == -2
    assert lib.pnp_prior_destroy(h) == 0


def test_struct_sizes_match_header(tmp_path):
    """Sizes and field offsets of the ABI structs: the C header as compiled
    by the host compiler (tests/host/abi_layout.cpp) against the ctypes
    binding."""
    import subprocess
    from paper_2411_01955_amd._lib import HQSOpts, HQSReport, Slice, Tuning
    exe = str(tmp_path / "abi_layout")
    src = os.path.join(ROOT, "tests", "host", "abi_layout.cpp")
    r = subprocess.run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([exe], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    structs = {"pnp_hqs_opts": HQSOpts, "pnp_hqs_report": HQSReport, "pnp_slice": Slice, "pnp_tuning": Tuning}
    for key, val in got.items():
        name, _, field = key.partition(".")
        T = structs[name]
        want = C.sizeof(T) if not field else getattr(T, {"lambda": "lam"}.get(field, field)).offset
        assert int(val) == want, (key, val, want)
