"""Pins of the oracle's coil sensitivity estimate (k-space centre, Hamming
window, root-sum-of-squares, mask) against numpy's FFT on a full Cartesian
grid, hand values of the window, and the exact recovery of the maps when
the window is flat and the k-space is fully sampled."""
import math

import numpy as np

import synth
from oracle import ndft, smaps


def test_hamming_window_values():
    c = 10.0
    h = smaps.hamming([0.0, c / 2, -c / 2, c, -c, c + 1e-9, 3 * c], c)
    # 0.54 + 0.46 cos(0) = 1; cos(pi/2) = 0 -> 0.54; cos(pi) = -1 -> 0.08; outside 0
    assert np.allclose(h, [1.0, 0.54, 0.54, 0.08, 0.08, 0.0, 0.0], atol=1e-15)


def _cartesian_data(n, L, x):
    S = synth.smaps2d(n, L).astype(np.complex128)
    S /= np.sqrt((np.abs(S) ** 2).sum(0))          # unit sum of squares in FP64
    k = synth.cartesian2d(n, np.float64)
    # y_l on the centred grid: fftshift(fft2(ifftshift(S_l x))) / n, kx fastest
    y = np.stack([(np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(S[l] * x))) / n).ravel() for l in range(L)])
    return S, k, y


def test_coil_images_equal_windowed_inverse_fft():
    """Cartesian full grid: z_l = n * fftshift(ifft2(ifftshift(H * Y_l))) with the
    separable window H[my, mx] = h(my) h(mx) on the integer frequencies."""
    n, L = 32, 3
    x = synth.white_complex((n, n), 71).astype(np.complex128)
    S, k, y = _cartesian_data(n, L, x)
    m = np.arange(n) - n // 2
    h = smaps.hamming(m, 6.0)
    H = np.outer(h, h)
    z = smaps.coil_images(y, k, (n, n), width=12.0)
    for l in range(L):
        Y = y[l].reshape(n, n)
        ref = n * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(H * Y)))
        assert np.abs(z[l] - ref).max() < 1e-12 * np.abs(ref).max()


def test_flat_window_full_sampling_recovers_maps():
    """With a flat window (huge width) and full Cartesian sampling the coil
    images are S_l x exactly; for a real positive object the normalised
    estimate is S_l itself (the maps have unit sum of squares)."""
    n, L = 32, 4
    yy, xx = np.mgrid[0:n, 0:n] - n / 2
    x = (1.0 + np.exp(-(xx ** 2 + yy ** 2) / (2 * (0.3 * n) ** 2))).astype(np.complex128)
    S, k, y = _cartesian_data(n, L, x)
    est, mask = smaps.estimate(y, k, (n, n), width=1e9, threshold=0.0)
    assert mask.all()
    assert np.abs(est - S).max() < 1e-10


def test_mask_and_unit_sum_of_squares():
    n, L = 32, 4
    x, _ = synth.phantom2d(n, 72)
    S, k, y = _cartesian_data(n, L, x.astype(np.complex128))
    est, mask = smaps.estimate(y, k, (n, n), width=20.0, threshold=0.2)
    z = smaps.coil_images(y, k, (n, n), width=20.0)
    s = np.sqrt((np.abs(z) ** 2).sum(0))
    assert np.array_equal(mask, s > 0.2 * s.max())
    assert 0 < mask.sum() < n * n
    assert np.all(est[:, ~mask] == 0)
    sos = np.sqrt((np.abs(est) ** 2).sum(0))
    assert np.abs(sos[mask] - 1.0).max() < 1e-12


def test_estimate_is_invariant_to_data_scale_up_to_phase():
    n, L = 32, 3
    x, _ = synth.phantom2d(n, 73)
    S, k, y = _cartesian_data(n, L, x.astype(np.complex128))
    a, _ = smaps.estimate(y, k, (n, n))
    c = 3.0 * np.exp(0.7j)
    b, _ = smaps.estimate(c * y, k, (n, n))
    assert np.abs(b - a * np.exp(0.7j)).max() < 1e-12
