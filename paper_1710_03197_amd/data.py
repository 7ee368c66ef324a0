"""Seeded synthetic inputs shaped like the paper's MRI workloads.

The paper's own data (a 3T brain template resized to 512x512 and a PROPELLER
k-space trajectory, Section 2.3) is not available, so every workload is built
here from a seed: analytic non-Cartesian trajectories (radial, golden-angle
radial, Fibonacci koosh-ball, variable-density spiral), ellipse/ellipsoid
phantoms, smooth Gaussian-bump coil sensitivities and complex Gaussian noise.

This module holds none of the transform's arithmetic: it only draws inputs.
Both the HIP path and the FP64 oracle consume its outputs, so it imports
neither of them.  Trajectories are built in float64 and then cast to float32
(radians, array shape [M, d], axis a of omega pairs with image axis a).
Images are complex64 in C order (last axis fastest).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_RATIO = (1.0 + math.sqrt(5.0)) / 2.0


# ---------------------------------------------------------------- trajectories
def radial_2d(n_spokes: int, n_read: int) -> np.ndarray:
    """Evenly spaced full-diameter spokes: theta_s = pi*s/n_spokes,
    r_j = -pi + 2*pi*j/n_read, sample m = s*n_read + j."""
    s = np.arange(n_spokes, dtype=np.float64)
    j = np.arange(n_read, dtype=np.float64)
    theta = np.pi * s / n_spokes
    r = -np.pi + 2.0 * np.pi * j / n_read
    om = np.empty((n_spokes, n_read, 2), dtype=np.float64)
    om[..., 0] = r[None, :] * np.cos(theta)[:, None]
    om[..., 1] = r[None, :] * np.sin(theta)[:, None]
    return om.reshape(-1, 2).astype(np.float32)


def golden_radial_2d(n_spokes: int, n_read: int) -> np.ndarray:
    """Golden-angle radial: theta_s = s*pi/phi (about 111.246 degrees apart),
    full diameters r_j = -pi + 2*pi*j/n_read."""
    s = np.arange(n_spokes, dtype=np.float64)
    j = np.arange(n_read, dtype=np.float64)
    theta = s * np.pi / GOLDEN_RATIO
    r = -np.pi + 2.0 * np.pi * j / n_read
    om = np.empty((n_spokes, n_read, 2), dtype=np.float64)
    om[..., 0] = r[None, :] * np.cos(theta)[:, None]
    om[..., 1] = r[None, :] * np.sin(theta)[:, None]
    return om.reshape(-1, 2).astype(np.float32)


def koosh_ball_3d(n_spokes: int, n_read: int) -> np.ndarray:
    """Centre-out 3D radial spokes on a Fibonacci sphere:
    z_s = 1 - (2s+1)/n_spokes, azimuth_s = s*pi*(3-sqrt(5)),
    r_j = pi*j/n_read (j = 0 .. n_read-1; every spoke starts at omega = 0)."""
    s = np.arange(n_spokes, dtype=np.float64)
    j = np.arange(n_read, dtype=np.float64)
    z = 1.0 - (2.0 * s + 1.0) / n_spokes
    az = s * np.pi * (3.0 - math.sqrt(5.0))
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([rho * np.cos(az), rho * np.sin(az), z], axis=-1)  # [S,3]
    r = np.pi * j / n_read
    om = r[None, :, None] * d[:, None, :]
    return om.reshape(-1, 3).astype(np.float32)


def spiral_2d(m: int, interleaves: int, turns: int) -> np.ndarray:
    """Archimedean variable-density spiral, m samples over `interleaves` arms:
    theta(t) = 2*pi*turns*t + 2*pi*l/interleaves, r(t) = pi*t^2, t in [0,1)
    evenly spaced per arm.  The first (m mod interleaves) arms get one extra
    sample so the total is exactly m."""
    base, extra = divmod(m, interleaves)
    parts = []
    for ell in range(interleaves):
        n = base + (1 if ell < extra else 0)
        t = np.arange(n, dtype=np.float64) / max(n, 1)
        theta = 2.0 * np.pi * turns * t + 2.0 * np.pi * ell / interleaves
        r = np.pi * t * t
        parts.append(np.stack([r * np.cos(theta), r * np.sin(theta)], axis=-1))
    return np.concatenate(parts, axis=0).astype(np.float32)


def perturb(om: np.ndarray, K, rng: np.random.Generator) -> np.ndarray:
    """Shift every coordinate by U(-1/2, 1/2) oversampled-grid cells
    (2*pi/K_a radians per cell) and wrap into [-pi, pi)."""
    om64 = om.astype(np.float64)
    K = np.asarray(K, dtype=np.float64)
    delta = rng.uniform(-0.5, 0.5, size=om64.shape) * (2.0 * np.pi / K)[None, :]
    w = om64 + delta
    w = (w + np.pi) % (2.0 * np.pi) - np.pi
    return w.astype(np.float32)


# -------------------------------------------------------------------- images
def _grid_coords(N):
    """Normalised field of view [-1, 1) per axis: p = (i - N/2)/(N/2)."""
    axes = [(np.arange(n, dtype=np.float64) - n // 2) / (n // 2) for n in N]
    return np.meshgrid(*axes, indexing="ij")


def random_complex_image(N, rng: np.random.Generator) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0, 1)."""
    shape = tuple(int(n) for n in N)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


def ellipse_phantom(N, n_ellipses: int, rng: np.random.Generator) -> np.ndarray:
    """Sum of filled ellipses (2D) or ellipsoids (3D) on [-1,1)^d: centres
    1.2*(U-1/2) per axis, semi-axes 0.05 + 0.45*U, rotation pi*U (2D) or three
    Euler angles 2*pi*U (3D), intensity U.  Returns float64 (real)."""
    d = len(N)
    P = np.stack(_grid_coords(N), axis=-1)  # [..., d]
    img = np.zeros(tuple(N), dtype=np.float64)
    for _ in range(n_ellipses):
        c = 1.2 * (rng.uniform(size=d) - 0.5)
        ax = 0.05 + 0.45 * rng.uniform(size=d)
        if d == 2:
            a = np.pi * rng.uniform()
            R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
        elif d == 3:
            a, b, g = 2.0 * np.pi * rng.uniform(size=3)
            Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
            Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
            Rx = np.array([[1, 0, 0], [0, math.cos(g), -math.sin(g)], [0, math.sin(g), math.cos(g)]])
            R = Rz @ Ry @ Rx
        else:
            R = np.eye(d)
        val = rng.uniform()
        Q = (P - c) @ R  # coordinates in the ellipse frame
        inside = np.sum((Q / ax) ** 2, axis=-1) <= 1.0
        img[inside] += val
    return img


def smooth_phase(N, rng: np.random.Generator) -> np.ndarray:
    """exp(i*pi*q(p)) with q a seeded quadratic polynomial in the normalised
    coordinates, every coefficient drawn from U(-1/2, 1/2)."""
    P = _grid_coords(N)
    d = len(N)
    q = np.full(P[0].shape, rng.uniform(-0.5, 0.5))
    for a in range(d):
        q += rng.uniform(-0.5, 0.5) * P[a]
    for a in range(d):
        for b in range(a, d):
            q += rng.uniform(-0.5, 0.5) * P[a] * P[b]
    return np.exp(1j * np.pi * q)


def coil_maps(N, n_coils: int, rng: np.random.Generator) -> np.ndarray:
    """Smooth complex sensitivities c_i(p) = exp(-|p - q_i|^2 / (2*0.6^2)) *
    exp(i*(alpha_i + gamma_i . p)), q_i on a radius-1.2 circle at angle
    2*pi*i/C plus a jitter of up to 0.2 rad (in the first two axes; 0 in any
    third axis).  Returns complex64 [C, *N]."""
    P = np.stack(_grid_coords(N), axis=-1)
    d = len(N)
    out = np.empty((n_coils,) + tuple(N), dtype=np.complex64)
    for i in range(n_coils):
        ang = 2.0 * np.pi * i / n_coils + rng.uniform(-0.2, 0.2)
        q = np.zeros(d)
        q[0] = 1.2 * math.cos(ang)
        if d > 1:
            q[1] = 1.2 * math.sin(ang)
        alpha = rng.uniform(0.0, 2.0 * np.pi)
        gamma = rng.uniform(-1.0, 1.0, size=d)
        mag = np.exp(-np.sum((P - q) ** 2, axis=-1) / (2.0 * 0.6 ** 2))
        out[i] = (mag * np.exp(1j * (alpha + P @ gamma))).astype(np.complex64)
    return out


def complex_noise(shape, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Real and imaginary parts each N(0, sigma^2)."""
    return (sigma * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)


# ------------------------------------------------------------------- configs
def config1(seed: int = 1) -> dict:
    """2D 64x64 random complex image, grid 128x128, J=6, 32 evenly spaced
    spokes x 128 readout points (M = 4096)."""
    rng = np.random.default_rng(seed)
    N, K = (64, 64), (128, 128)
    return dict(name="2d_64_radial", d=2, N=N, K=K, J=6, om=radial_2d(32, 128),
                x=random_complex_image(N, rng))


def config2(seed: int = 2, n_spokes: int = 256, n_read: int = 512, N=(256, 256)) -> dict:
    """2D 256x256 ellipse phantom (10 ellipses) with a smooth random phase,
    grid 512x512, J=6, golden-angle radial 256 spokes x 512 readout
    (M = 131072), y = A x + complex noise of sigma 1e-3 is formed by the
    caller (it needs the forward transform)."""
    rng = np.random.default_rng(seed)
    N = tuple(N)
    K = tuple(2 * n for n in N)
    x = (ellipse_phantom(N, 10, rng) * smooth_phase(N, rng)).astype(np.complex64)
    return dict(name="2d_256_golden_radial", d=2, N=N, K=K, J=6,
                om=golden_radial_2d(n_spokes, n_read), x=x, noise_rng=rng)


def config3(seed: int = 3, n_spokes: int = 8192, n_read: int = 256, N=(128, 128, 128)) -> dict:
    """3D 128^3 real ellipsoid phantom (12 ellipsoids), grid 256^3, J=6,
    koosh-ball radial 8192 spokes x 256 readout (M = 2,097,152)."""
    rng = np.random.default_rng(seed)
    N = tuple(N)
    K = tuple(2 * n for n in N)
    x = ellipse_phantom(N, 12, rng).astype(np.complex64)
    return dict(name="3d_128_koosh", d=3, N=N, K=K, J=6,
                om=koosh_ball_3d(n_spokes, n_read), x=x)


def config4(seed: int = 4, n_problems: int = 24, n_coils: int = 8,
            sizes=(128, 192, 256, 320, 384), m_range=(20000, 200000)) -> list:
    """Uneven batch: per problem N drawn from `sizes` (square), sigma = 2,
    J = 6, M ~ U{m_range}, spiral with interleaves and turns ~ U{8..32},
    `n_coils` Gaussian-bump coil maps and a random complex image."""
    rng = np.random.default_rng(seed)
    probs = []
    for p in range(n_problems):
        n = int(rng.choice(sizes))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        L = int(rng.integers(8, 33))
        T = int(rng.integers(8, 33))
        N = (n, n)
        probs.append(dict(name=f"spiral_{p}", d=2, N=N, K=(2 * n, 2 * n), J=6,
                          om=spiral_2d(m, L, T), coils=coil_maps(N, n_coils, rng),
                          x=random_complex_image(N, rng)))
    return probs


def config5(seed: int = 5, n_coils: int = 4, n_spokes: int = 128, n_read: int = 512,
            N=(256, 256)) -> dict:
    """Differentiation workload: 2D 256x256, grid 512x512, J=6, 4 coils,
    golden-angle radial 128 x 512 (M = 65536) with a +-0.5-cell seeded
    perturbation; x is an ellipse phantom, the target comes from a second,
    independently drawn ellipse phantom."""
    rng = np.random.default_rng(seed)
    N = tuple(N)
    K = tuple(2 * n for n in N)
    om = perturb(golden_radial_2d(n_spokes, n_read), K, rng)
    x = (ellipse_phantom(N, 10, rng) * smooth_phase(N, rng)).astype(np.complex64)
    x_target = (ellipse_phantom(N, 10, rng) * smooth_phase(N, rng)).astype(np.complex64)
    coils = coil_maps(N, n_coils, rng)
    return dict(name="2d_256_grad", d=2, N=N, K=K, J=6, om=om, x=x, x_target=x_target,
                coils=coils)
