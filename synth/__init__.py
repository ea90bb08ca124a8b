"""Seeded synthetic workload generators (inputs only).

This module produces the *inputs* of the reconstruction problem: phantoms,
coil sensitivity maps, non-Cartesian trajectories, density-compensation
weights, complex Gaussian noise and the uneven multi-slice table.  It holds
none of the method's arithmetic (no Fourier operator, no solver, no prior):
both the FP64 oracle and the GPU library consume what it returns, so the two
sides always work on bit-identical inputs.

Conventions shared by every generator
* Images are ``[ny][nx]`` (or ``[nz][ny][nx]``), x fastest.  Pixel index ``i``
  maps to the normalised coordinate ``u = (i - n/2)/n`` in ``[-1/2, 1/2)``;
  the field of view (FOV) is 1 in these units.
* Trajectories are ``float32`` arrays ``[M][d]`` ordered ``(kx, ky[, kz])``
  in radians per pixel, inside ``[-pi, pi]``.
* Complex arrays are returned as ``complex64`` (what the GPU consumes); the
  oracle promotes the very same values to ``complex128``.
* Every function takes an explicit integer seed and uses
  ``numpy.random.default_rng(seed)``.

The acquisition follows the paper's simulation set-up (Sec. 4.1): a spiral
(or radial) non-Cartesian pattern at a given acceleration factor, additive
white Gaussian k-space noise whose variance is 1e-4 times the maximum over
pixels of the coil-summed squared magnitude, and smooth complex coil maps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0

# Seed bases (stated recipe): phantom i -> 1000 + i, noise i -> 2000 + i,
# training phantoms 0..1999, held-out phantoms 10000..10099.
SEED_PHANTOM = 1000
SEED_NOISE = 2000
SEED_TRAIN = 0
SEED_HELDOUT = 10000


def _coords(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - n / 2) / n


# ---------------------------------------------------------------- phantoms
def phantom2d(n: int, seed: int, n_ellipses: int = 8):
    """Random-ellipse complex phantom of shape ``[n][n]``.

    Ellipse 0 is an outer "head" (semi-axes U(0.75, 0.9)*FOV/2, centre
    within +-0.05 FOV); ellipses 1.. have centres U(-0.5, 0.5)*FOV/2,
    semi-axes U(0.05, 0.35)*FOV/2, angles U(0, pi) and magnitudes U(0.1, 1),
    painted in order (later ones overwrite).  A smooth phase exp(i*phi), phi a
    random quadratic polynomial with max |phi| <= pi/2, multiplies the image.

    Returns ``(x complex64 [n][n], support bool [n][n])``.
    """
    rng = np.random.default_rng(seed)
    u = _coords(n)
    Y, X = np.meshgrid(u, u, indexing="ij")
    mag = np.zeros((n, n))
    support = np.zeros((n, n), dtype=bool)
    for e in range(n_ellipses):
        if e == 0:
            a, b = rng.uniform(0.75, 0.9, 2) * 0.5
            cx, cy = rng.uniform(-0.05, 0.05, 2)
        else:
            cx, cy = rng.uniform(-0.5, 0.5, 2) * 0.5
            a, b = rng.uniform(0.05, 0.35, 2) * 0.5
        th = rng.uniform(0.0, math.pi)
        val = rng.uniform(0.1, 1.0)
        c, s = math.cos(th), math.sin(th)
        xr = (X - cx) * c + (Y - cy) * s
        yr = -(X - cx) * s + (Y - cy) * c
        inside = (xr / a) ** 2 + (yr / b) ** 2 <= 1.0
        mag[inside] = val
        support |= inside
    coef = rng.uniform(-1.0, 1.0, 6)
    phi = (coef[0] + coef[1] * X + coef[2] * Y + coef[3] * X * X
           + coef[4] * X * Y + coef[5] * Y * Y)
    peak = np.abs(phi).max()
    phi *= (math.pi / 2) * rng.uniform(0.3, 1.0) / max(peak, 1e-12)
    x = mag * np.exp(1j * phi)
    return x.astype(np.complex64), support


def phantom3d(n: int, seed: int, n_ellipsoids: int = 8):
    """3D analogue of :func:`phantom2d` (ellipsoids, ``[n][n][n]``)."""
    rng = np.random.default_rng(seed)
    u = _coords(n)
    Z, Y, X = np.meshgrid(u, u, u, indexing="ij")
    mag = np.zeros((n, n, n), dtype=np.float32)
    support = np.zeros((n, n, n), dtype=bool)
    for e in range(n_ellipsoids):
        if e == 0:
            ax = rng.uniform(0.75, 0.9, 3) * 0.5
            cen = rng.uniform(-0.05, 0.05, 3)
        else:
            cen = rng.uniform(-0.5, 0.5, 3) * 0.5
            ax = rng.uniform(0.05, 0.35, 3) * 0.5
        # random rotation about z then x
        t1, t2 = rng.uniform(0.0, math.pi, 2)
        val = rng.uniform(0.1, 1.0)
        c1, s1, c2, s2 = math.cos(t1), math.sin(t1), math.cos(t2), math.sin(t2)
        dx, dy, dz = X - cen[0], Y - cen[1], Z - cen[2]
        xr = dx * c1 + dy * s1
        yr = -dx * s1 + dy * c1
        yr2 = yr * c2 + dz * s2
        zr = -yr * s2 + dz * c2
        inside = (xr / ax[0]) ** 2 + (yr2 / ax[1]) ** 2 + (zr / ax[2]) ** 2 <= 1.0
        mag[inside] = val
        support |= inside
    coef = rng.uniform(-1.0, 1.0, 4)
    phi = coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z
    peak = np.abs(phi).max()
    phi *= (math.pi / 2) * rng.uniform(0.3, 1.0) / max(peak, 1e-12)
    x = mag * np.exp(1j * phi)
    return x.astype(np.complex64), support


# ------------------------------------------------------------ coil maps
def smaps2d(n: int, L: int):
    """Gaussian coil profiles centred on a circle of radius 0.6*FOV at angles
    2*pi*l/L, width (std) 0.5*FOV, phase exp(i*2*pi*l/L), normalised so that
    the sum of squares over coils is 1 at every pixel.  ``[L][n][n]``."""
    u = _coords(n)
    Y, X = np.meshgrid(u, u, indexing="ij")
    maps = np.empty((L, n, n), dtype=np.complex128)
    for l in range(L):
        ang = 2 * math.pi * l / L
        cx, cy = 0.6 * math.cos(ang), 0.6 * math.sin(ang)
        g = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 0.5 ** 2))
        maps[l] = g * np.exp(1j * ang)
    sos = np.sqrt((np.abs(maps) ** 2).sum(0))
    return (maps / sos).astype(np.complex64)


def fibonacci_sphere(P: int, hemisphere: bool = False) -> np.ndarray:
    """``P`` nearly uniform unit vectors (Fibonacci lattice)."""
    i = np.arange(P, dtype=np.float64) + 0.5
    if hemisphere:
        z = 1.0 - i / P
    else:
        z = 1.0 - 2.0 * i / P
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (2 * math.pi / GOLDEN ** 2)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def smaps3d(n: int, L: int):
    """3D coil maps: Gaussian profiles centred on a Fibonacci sphere of radius
    0.6*FOV, width 0.5*FOV, phase exp(i*2*pi*l/L), SoS-normalised."""
    u = _coords(n).astype(np.float32)
    Z, Y, X = np.meshgrid(u, u, u, indexing="ij")
    cen = 0.6 * fibonacci_sphere(L)
    maps = np.empty((L, n, n, n), dtype=np.complex64)
    for l in range(L):
        g = np.exp(-((X - cen[l, 0]) ** 2 + (Y - cen[l, 1]) ** 2
                     + (Z - cen[l, 2]) ** 2) / (2 * 0.5 ** 2))
        maps[l] = g * np.complex64(np.exp(1j * 2 * math.pi * l / L))
    sos = np.sqrt((np.abs(maps) ** 2).sum(0))
    maps /= sos
    return maps


# --------------------------------------------------------- trajectories
@dataclass(frozen=True)
class Trajectory:
    """Sample coordinates plus the readout structure (for the DCF rule)."""
    k: np.ndarray          # float32 [M][d], radians per pixel
    n_readouts: int        # spokes / interleaves
    samples: int           # samples per readout (readout-major order)
    kind: str


def radial2d(spokes: int, S: int) -> Trajectory:
    """Golden-angle radial: spoke j at angle j*pi/golden, samples
    t_s = pi*(2s/S - 1), s = 0..S-1 (readout-major)."""
    j = np.arange(spokes, dtype=np.float64)[:, None]
    s = np.arange(S, dtype=np.float64)[None, :]
    t = math.pi * (2 * s / S - 1)
    th = j * math.pi / GOLDEN
    k = np.stack([t * np.cos(th), t * np.sin(th)], axis=-1).reshape(-1, 2)
    return Trajectory(k.astype(np.float32), spokes, S, "radial")


def spiral2d(interleaves: int, S: int) -> Trajectory:
    """Variable-density spiral: interleaf j of I, sample s of S, t = s/S,
    radius pi*t^1.5, angle 2*pi*(0.75*t + j/I)."""
    j = np.arange(interleaves, dtype=np.float64)[:, None]
    t = np.arange(S, dtype=np.float64)[None, :] / S
    r = math.pi * t ** 1.5
    th = 2 * math.pi * (0.75 * t + j / interleaves)
    k = np.stack([r * np.cos(th), r * np.sin(th)], axis=-1).reshape(-1, 2)
    return Trajectory(k.astype(np.float32), interleaves, S, "spiral")


def kooshball3d(spokes: int, S: int) -> Trajectory:
    """3D radial 'kooshball': full-diameter spokes along Fibonacci
    hemisphere directions, samples t_s = pi*(2s/S - 1)."""
    d = fibonacci_sphere(spokes, hemisphere=True)
    t = math.pi * (2 * np.arange(S, dtype=np.float64) / S - 1)
    k = (d[:, None, :] * t[None, :, None]).reshape(-1, 3)
    return Trajectory(k.astype(np.float32), spokes, S, "kooshball")


def cartesian2d(n: int, dtype=np.float32) -> np.ndarray:
    """Full Cartesian grid k = 2*pi*m/n, m = -n/2..n/2-1 ([n*n][2]),
    row-major in (ky, kx) with kx fastest."""
    m = 2 * math.pi * (np.arange(n) - n // 2) / n
    KY, KX = np.meshgrid(m, m, indexing="ij")
    return np.stack([KX.ravel(), KY.ravel()], axis=1).astype(dtype)


# ------------------------------------------------------------------ DCF
def voronoi_dcf(traj: Trajectory, n: int) -> np.ndarray:
    """Voronoi density-compensation weights for a 2D trajectory.

    Coincident samples are merged and share their cell area equally.  Cells
    that are unbounded, or reach beyond the sampled disk by more than one
    readout step, take the area of their inward neighbour on the same
    readout.  Normalised as ``w = area * N / (2*pi)^2`` so that a full
    Cartesian grid would give w = 1.  Returns float32 ``[M]``.
    """
    from scipy.spatial import Voronoi

    k = traj.k.astype(np.float64)
    M = k.shape[0]
    uniq, inv, counts = np.unique(k, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    vor = Voronoi(uniq)
    rad = np.linalg.norm(k, axis=1)
    step = np.median(np.linalg.norm(np.diff(k.reshape(traj.n_readouts, traj.samples, 2), axis=1), axis=2))
    rmax = rad.max() + step
    area_u = np.full(len(uniq), np.nan)
    for p, reg_idx in enumerate(vor.point_region):
        reg = vor.regions[reg_idx]
        if len(reg) == 0 or -1 in reg:
            continue
        poly = vor.vertices[reg]
        if np.linalg.norm(poly, axis=1).max() > rmax:
            continue
        x, y = poly[:, 0], poly[:, 1]
        area_u[p] = 0.5 * abs(np.dot(x, np.roll(y, 1)) - np.dot(y, np.roll(x, 1)))
    area = area_u[inv] / counts[inv]
    # fill outer/unbounded cells from the inward neighbour on the same readout
    a2 = area.reshape(traj.n_readouts, traj.samples)
    r2 = rad.reshape(traj.n_readouts, traj.samples)
    for j in range(traj.n_readouts):
        order = np.argsort(r2[j], kind="stable")
        last = None
        for s in order:
            if np.isnan(a2[j, s]):
                a2[j, s] = last if last is not None else 0.0
            last = a2[j, s]
    w = a2.reshape(-1) * (n * n) / (2 * math.pi) ** 2
    return w.astype(np.float32)


def radial3d_dcf(traj: Trajectory, n: int) -> np.ndarray:
    """Analytic density compensation for a full-diameter 3D radial pattern:
    each sample owns a share of the spherical shell it lies on (2 samples of
    every spoke per shell), the centre samples share the central ball.
    Normalised like :func:`voronoi_dcf` (``N/(2*pi)^3``)."""
    k = traj.k.astype(np.float64)
    r = np.linalg.norm(k, axis=1)
    dk = 2 * math.pi / traj.samples
    P = traj.n_readouts
    vol = 4 * math.pi * r ** 2 * dk / (2 * P)
    centre = r < 0.5 * dk
    vol[centre] = (4.0 / 3.0) * math.pi * (dk / 2) ** 3 / P
    return (vol * n ** 3 / (2 * math.pi) ** 3).astype(np.float32)


# ---------------------------------------------------------------- noise
def noise_variance(x: np.ndarray, smaps: np.ndarray) -> float:
    """nu = 1e-4 * max over pixels of sum_l |S_l x|^2 (image-domain maximum)."""
    xs = smaps.astype(np.complex128) * x.astype(np.complex128)[None]
    return 1e-4 * float((np.abs(xs) ** 2).sum(0).max())


def complex_noise(shape, nu: float, seed: int) -> np.ndarray:
    """Circular complex Gaussian noise CN(0, nu): real and imaginary parts
    independent with variance nu/2 each.  complex64."""
    rng = np.random.default_rng(seed)
    sd = math.sqrt(nu / 2)
    e = rng.standard_normal(shape) * sd + 1j * rng.standard_normal(shape) * sd
    return e.astype(np.complex64)


def white_complex(shape, seed: int) -> np.ndarray:
    """Unit-variance circular complex Gaussian test vector (complex64)."""
    rng = np.random.default_rng(seed)
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
            / math.sqrt(2)).astype(np.complex64)


# ------------------------------------------------------- anneal schedule
def geometric_sigmas(sigma0: float, sigma_end: float, n_out: int) -> np.ndarray:
    """sigma_k = sigma0 * xi^(k-1), k = 1..n_out, with xi chosen so that the
    last value is sigma_end (the annealing rule of Sec. 3.3 with the
    exponent read as k-1).  float64 [n_out]."""
    if n_out == 1:
        return np.array([sigma0], dtype=np.float64)
    xi = (sigma_end / sigma0) ** (1.0 / (n_out - 1))
    return sigma0 * xi ** np.arange(n_out, dtype=np.float64)


# ------------------------------------------------------- workload configs
@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    ndim: int
    L: int
    traj: Trajectory
    dcf: bool
    n_out: int
    n_cg: int
    sigma0: float
    sigma_end: float


def config_tiny() -> Workload:
    """64x64, 4 coils, 16 golden-angle spokes x 128 samples, no DCF,
    20 HQS iterations x 3 CG steps."""
    return Workload("tiny-64x64-L4-radial16x128", 64, 2, 4, radial2d(16, 128),
                    False, 20, 3, 0.1, 0.005)


def config_clinical() -> Workload:
    """320x320, 16 coils, VD spiral 32 x 400 (AF 8), Voronoi DCF,
    30 HQS iterations x 5 CG steps, sigma 0.1 -> 0.005."""
    return Workload("clinical-320x320-L16-spiral32x400", 320, 2, 16, spiral2d(32, 400),
                    True, 30, 5, 0.1, 0.005)


def config_3d(n: int = 128, L: int = 32, spokes: int = 4096, S: int = 256) -> Workload:
    """128^3, 32 coils, kooshball 4096 x 256, 20 HQS iterations x 5 CG."""
    return Workload(f"3d-{n}cube-L{L}-koosh{spokes}x{S}", n, 3, L, kooshball3d(spokes, S),
                    True, 20, 5, 0.1, 0.005)


def batched_slice_table(count: int = 24):
    """Uneven multi-slice table: slice i has n = (256, 320, 384)[i % 3],
    L = (8, 16, 32)[(i // 3) % 3], AF = (4, 8, 16)[(i // 9) % 3]; even i is
    golden-angle radial with S = 2n samples and round(N/(AF*S)) spokes, odd i
    a VD spiral with S = round(1.25 n) and round(N/(AF*S)) interleaves."""
    out = []
    for i in range(count):
        n = (256, 320, 384)[i % 3]
        L = (8, 16, 32)[(i // 3) % 3]
        af = (4, 8, 16)[(i // 9) % 3]
        out.append(dict(index=i, n=n, L=L, af=af, traj=uneven_slice_traj(n, af, i % 2 == 0)))
    return out


def uneven_slice_traj(n: int, af: int, radial: bool) -> Trajectory:
    """The trajectory rule of the uneven multi-slice table: golden-angle
    radial with S = 2n samples and round(N/(AF*S)) spokes, or a VD spiral with
    S = round(1.25 n) samples and round(N/(AF*S)) interleaves (N = n^2)."""
    N = n * n
    if radial:
        S = 2 * n
        return radial2d(max(1, round(N / (af * S))), S)
    S = round(1.25 * n)
    return spiral2d(max(1, round(N / (af * S))), S)


# ------------------------------------------------------ denoiser training data
def he_normal(shapes: dict, seed: int, last_scale: dict | None = None) -> dict:
    """Seeded He-normal weights for {name: (weight shape, bias shape)}:
    W ~ N(0, 2 / fan_in) with fan_in = prod(weight shape[1:]), biases zero;
    `last_scale` multiplies the named layers' weights.  Float32 values."""
    rng = np.random.default_rng(seed)
    out = {}
    for name in shapes:
        ws, bs = shapes[name]
        fan_in = int(np.prod(ws[1:]))
        w = rng.standard_normal(ws) * math.sqrt(2.0 / fan_in)
        w *= (last_scale or {}).get(name, 1.0)
        out[name] = (w.astype(np.float32).astype(np.float64), np.zeros(bs))
    return out


def denoise_pairs(images: np.ndarray, sigma_lo: float, sigma_hi: float, seed: int):
    """Noisy copies of `images` [B, H, W] complex: sigma_b ~ U(lo, hi) per
    image, independent N(0, sigma_b^2) noise on the real and imaginary parts.
    Returns (noisy complex64, sigma float32 [B])."""
    rng = np.random.default_rng(seed)
    B = images.shape[0]
    sig = rng.uniform(sigma_lo, sigma_hi, B).astype(np.float32)
    n = rng.standard_normal((2,) + images.shape)
    noisy = images + sig[:, None, None] * (n[0] + 1j * n[1])
    return noisy.astype(np.complex64), sig
