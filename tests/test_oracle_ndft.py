"""Pins of the exact NDFT oracle (Eq. 1) against facts it does not compute
itself: a dense matrix built entry by entry, numpy's FFT on a full Cartesian
grid, Parseval, the adjoint identity, and an independent KB-gridding
implementation whose deviation must match the closed-form alias error."""
import math

import numpy as np
import pytest

import synth
from oracle import ndft, gridding


def _rand_traj(M, d, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-math.pi, math.pi, (M, d)).astype(np.float32)


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (4, 4, 4)])
def test_forward_equals_dense_matrix(shape):
    L, M = 2, 20
    rng = np.random.default_rng(1)
    x = synth.white_complex(shape, 3)
    S = synth.white_complex((L,) + shape, 4)
    k = _rand_traj(M, len(shape), 5)
    A = ndft.dense_matrix(shape, S, k)
    y_dense = (A @ x.astype(np.complex128).ravel()).reshape(L, M)
    y = ndft.forward(x, S, k)
    assert np.max(np.abs(y - y_dense)) <= 1e-13 * np.max(np.abs(y_dense)) * 10
    # adjoint = conjugate transpose of the same dense matrix (with weights)
    yv = synth.white_complex((L, M), 6)
    w = rng.uniform(0.5, 2.0, M)
    x_dense = (A.conj().T @ (yv.astype(np.complex128) * w[None]).ravel()).reshape(shape)
    xa = ndft.adjoint(yv, S, k, w)
    assert np.max(np.abs(xa - x_dense)) <= 1e-12 * np.max(np.abs(x_dense))


@pytest.mark.parametrize("n", [8, 16, 12])
def test_cartesian_full_grid_equals_fft(n):
    x = synth.white_complex((n, n), 7)
    k = synth.cartesian2d(n, np.float64)
    y = ndft.forward(x, np.ones((1, n, n), np.complex64), k)[0].reshape(n, n)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x.astype(np.complex128)))) / n
    assert np.max(np.abs(y - ref)) <= 1e-12
    # inverse direction: the adjoint is numpy's inverse FFT (unitary scale)
    xa = ndft.adjoint(y.reshape(1, -1), np.ones((1, n, n), np.complex64), k)
    assert np.max(np.abs(xa - x)) <= 1e-12


def test_parseval_and_identity_normal_with_sos_maps():
    n, L = 16, 4
    x = synth.white_complex((n, n), 8).astype(np.complex128)
    S = synth.smaps2d(n, L)
    k = synth.cartesian2d(n, np.float64)
    y = ndft.forward(x, S, k)
    # sum_l ||F S_l x||^2 = sum_l ||S_l x||^2 = ||x||^2 (SoS = 1, up to f32 rounding of S)
    sos = (np.abs(S.astype(np.complex128)) ** 2).sum(0)
    assert abs(np.linalg.norm(y) ** 2 - np.sum(sos * np.abs(x) ** 2)) <= 1e-10 * np.linalg.norm(x) ** 2
    xn = ndft.normal(x, S, k)
    assert np.max(np.abs(xn - sos * x)) <= 1e-12
    assert np.max(np.abs(sos - 1)) < 1e-6


@pytest.mark.parametrize("d", [2, 3])
def test_adjoint_identity(d):
    shape = (12, 10) if d == 2 else (6, 8, 4)
    L, M = 3, 150
    x = synth.white_complex(shape, 9)
    S = synth.white_complex((L,) + shape, 10)
    k = _rand_traj(M, d, 11)
    y = synth.white_complex((L, M), 12)
    w = np.random.default_rng(0).uniform(0.1, 3, M)
    lhs = np.vdot(ndft.forward(x, S, k) * w, y)
    rhs = np.vdot(x.astype(np.complex128), ndft.adjoint(y, S, k, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_sampled_evaluations_match_full():
    n, L, M = 12, 2, 64
    x = synth.white_complex((n, n), 13)
    S = synth.white_complex((L, n, n), 14)
    k = _rand_traj(M, 2, 15)
    y = synth.white_complex((L, M), 16)
    w = np.random.default_rng(1).uniform(0.5, 1.5, M)
    idx = np.array([0, 5, 63, 17])
    assert np.allclose(ndft.forward_at(x, S, k, idx), ndft.forward(x, S, k)[:, idx], atol=1e-13)
    pix = np.array([0, 7, 143, 60])
    full = ndft.adjoint(y, S, k, w).ravel()[pix]
    assert np.allclose(ndft.adjoint_at(y, S, k, w, pix), full, atol=1e-12)
    # 3D
    sh = (4, 6, 8)
    x3 = synth.white_complex(sh, 17)
    S3 = synth.white_complex((2,) + sh, 18)
    k3 = _rand_traj(40, 3, 19)
    y3 = synth.white_complex((2, 40), 20)
    pix3 = np.array([0, 33, 191])
    assert np.allclose(ndft.adjoint_at(y3, S3, k3, None, pix3), ndft.adjoint(y3, S3, k3).ravel()[pix3], atol=1e-12)


def test_kb_response_closed_form_vs_poisson():
    # the Poisson tail decays like 1/P: Richardson-extrapolate P -> infinity
    K = 64
    for r, g in [(0, 0.0), (-16, 3.3), (15, -7.71), (-32 // 2, 0.5)]:
        a = gridding.response_1d(np.array(r, float), np.array(g), K)
        b1 = gridding.response_poisson_1d(r, g, K, P=100000)
        b2 = gridding.response_poisson_1d(r, g, K, P=200000)
        assert abs(a - (2 * b2 - b1)) < 1e-12
        assert abs(a - 1) > 1e-7      # the alias error itself is not negligible


def test_beatty_beta_value():
    assert abs(gridding.beatty_beta(6, 2) - 13.8551) < 1e-4


@pytest.mark.parametrize("n", [32, 48])
def test_kb_gridding_error_matches_prediction(n):
    """Two independent operators (exact NDFT, FP64 KB gridding) differ by
    the closed-form KB alias error: a dropped term, a wrong sign or a wrong
    index in either would show up as an O(1) discrepancy."""
    M = 3000
    k = _rand_traj(M, 2, 21)
    x = synth.white_complex((n, n), 22)
    S = np.ones((1, n, n), np.complex64)
    y_ex = ndft.forward(x, S, k)
    kb = gridding.KBGridding((n, n), k)
    y_kb = kb.forward(x, S)
    rel = np.linalg.norm(y_kb - y_ex) / np.linalg.norm(y_ex)
    pred = gridding.predicted_rel_rms_white(n, 2)
    assert pred / 2 < rel < pred * 2, (rel, pred)
    assert rel < 2e-5
    # and the adjoint
    yv = synth.white_complex((1, M), 23)
    x_ex = ndft.adjoint(yv, S, k)
    x_kb = kb.adjoint(yv, S)
    rel_a = np.linalg.norm(x_kb - x_ex) / np.linalg.norm(x_ex)
    assert rel_a < 3 * pred


def test_predicted_kb_error_level():
    # Kaiser-Bessel aliasing level for W = 6, oversampling 2 (Beatty shape): about 6.7e-6 rel-RMS in 2D
    p = gridding.predicted_rel_rms_white(320, 2)
    assert 3e-6 < p < 1.2e-5
