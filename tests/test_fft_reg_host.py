"""CPU check of the GPU library's register DFTs (fft_reg.hpp): a host
harness built from the same header computes every DFT size and four-step
factorisation the kernels use; numpy's FFT is the reference."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_01955_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host", "fft_reg_check.cpp")


@pytest.fixture(scope="module")
def rows(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("fftreg") / "fft_reg_check")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "-O2", "-std=c++17", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        pytest.fail(r.stderr[-3000:])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    res = []
    for line in out.strip().splitlines():
        f = line.split()
        kind, n, inv = f[0], int(f[1]), int(f[2])
        vals = np.array(f[3:], dtype=np.float64)
        c = vals[0::2] + 1j * vals[1::2]
        res.append((kind, n, inv, c[:n], c[n:]))
    return res


def test_toeplitz_column_chain(rows):
    """FFT -> multiply by real T -> the kernel's transposed inverse FFT equals
    K * ifft(T * fft(x)) (the unnormalised inverse)."""
    seen = []
    for kind, n, inv, x, rest in rows:
        if kind != "toep":
            continue
        T = rest[:n].real
        Y = rest[n:]
        ref = np.fft.ifft(T * np.fft.fft(x)) * n
        assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 5e-7, n
        seen.append(n)
    assert sorted(seen) == [128, 640, 768, 1024]


def test_register_dfts_match_numpy(rows):
    seen = set()
    for kind, n, inv, x, X in rows:
        if kind == "toep":
            continue
        ref = np.fft.ifft(x) * n if inv else np.fft.fft(x)
        err = np.linalg.norm(X - ref) / np.linalg.norm(ref)
        assert err < 3e-7, (kind, n, inv, err)
        seen.add((kind, n))
    for n in (2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32):
        assert ("dft", n) in seen
    for K in (128, 192, 256, 512, 640, 768, 1024):
        assert ("four", K) in seen
    for n in (16, 32):                     # middle half zero: the padded forward lines
        assert ("hz", n) in seen
