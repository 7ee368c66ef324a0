"""Pins of the oracle's sampling-density compensation (paper Section 2.2,
"Density compensation and gridding", Eq. pipe_density, after Pipe and Menon)
against facts that do not come from the oracle.

The printed iteration w <- w / (A A^H w) (density_compensation_aah):
- one step equals 1 / |E E^H 1| (modulus reading) and 1 / (E E^H 1) (complex
  reading), E the brute-force NUDFT matrix, within the NUFFT's own error;
- a modulus step is scale invariant;
- measured in float64 on an evenly spaced radial trajectory, the map does not
  settle: its fixed-point residual and the spread of the weights grow over the
  iterations, while the V V^H reading on the same trajectory approaches its
  fixed point monotonically.  This is the fact the GPU library's choice of
  V V^H rests on.

The reading w <- w / V V^H w (density_compensation_vvh):

- a dense interpolation matrix V built here from scipy's I0 and Beatty's
  beta (not the oracle's kernel code): one step equals 1 / (V V^T 1);
- a full Cartesian set of frequencies sees the same neighbourhood at every
  sample, so the weights are uniform, with the value from the dense V;
- scale invariance of a step (w -> c w gives the same next iterate);
- convergence towards the fixed point V V^H w = 1;
- on a radial trajectory the weights grow with the distance from the centre
  (the density of radial samples falls as 1/|k|).
"""
import math

import numpy as np
import scipy.special

from nudft import nudft_adjoint, nudft_forward, rel_l2
from paper_1710_03197_amd import data


def _dense_V(om, K, J):
    """V[m, k] = prod_a phi(u_ma - k_a) over the J taps k_a = k0 + j (mod K),
    phi(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta) (peak 1),
    beta = pi sqrt((J/s)^2 (s-1/2)^2 - 0.8)
    with s = 2; k0 = floor(u - J/2) + 1, u = omega K / (2 pi)."""
    om = np.asarray(om, np.float64)
    M, d = om.shape
    beta = math.pi * math.sqrt((J / 2.0) ** 2 * 1.5 ** 2 - 0.8)
    V = np.zeros((M,) + tuple(K))
    for m in range(M):
        per_axis = []
        for a in range(d):
            u = om[m, a] * (K[a] / (2.0 * math.pi))
            k0 = math.floor(u - J / 2.0) + 1
            row = np.zeros(K[a])
            for j in range(J):
                t = u - (k0 + j)
                row[(k0 + j) % K[a]] += (scipy.special.i0(beta * math.sqrt(max(0.0, 1.0 - (2.0 * t / J) ** 2)))
                                         / scipy.special.i0(beta))
            per_axis.append(row)
        outer = per_axis[0]
        for r in per_axis[1:]:
            outer = np.multiply.outer(outer, r)
        V[m] = outer
    return V.reshape(M, -1)


def test_one_step_against_dense_interpolator(orc):
    N, K = (6, 8), (12, 16)
    om = np.random.default_rng(4).uniform(-np.pi, np.pi, (60, 2)).astype(np.float32)
    V = _dense_V(om, K, 6)
    ref = 1.0 / (V @ (V.T @ np.ones(60)))
    assert rel_l2(orc.density_compensation_vvh(om, N, K, 6, 1), ref) < 1e-12


def test_cartesian_weights_are_uniform(orc):
    """Frequencies 2 pi (k + 1/4) / 8 put every sample half-way between grid
    points of the 16-point grid (u = 2k + 1/2, clear of the window tie-break)
    and the set is invariant under a shift by 2 grid cells, so every sample
    has the same neighbourhood: uniform weights up to the float32 rounding of
    omega (~1e-7)."""
    N, K = (8, 8), (16, 16)
    k = np.stack(np.meshgrid(np.arange(-4, 4), np.arange(-4, 4), indexing="ij"), -1).reshape(-1, 2)
    om = (2 * np.pi * (k + 0.25) / 8.0).astype(np.float32)
    V = _dense_V(om, K, 6)
    ref = 1.0 / (V @ (V.T @ np.ones(len(om))))
    assert np.ptp(ref) <= 1e-6 * ref.mean()
    for iters in (1, 4):
        w = orc.density_compensation_vvh(om, N, K, 6, iters)
        assert np.ptp(w) <= 1e-6 * w.mean()
    assert rel_l2(orc.density_compensation_vvh(om, N, K, 6, 1), ref) < 1e-12


def test_step_is_scale_invariant(orc):
    N, K = (16,), (32,)
    om = np.random.default_rng(1).uniform(-np.pi, np.pi, (50, 1)).astype(np.float32)
    w0 = np.random.default_rng(2).uniform(0.5, 1.5, 50)
    a = orc.density_compensation_vvh(om, N, K, 6, 1, w0)
    b = orc.density_compensation_vvh(om, N, K, 6, 1, 7.5 * w0)
    assert rel_l2(a, b) < 1e-12


def test_iterations_approach_the_fixed_point(orc):
    N, K = (24, 24), (48, 48)
    om = data.golden_radial_2d(20, 48)
    V = _dense_V(om, K, 6)
    res = []
    for iters in (1, 5, 20):
        w = orc.density_compensation_vvh(om, N, K, 6, iters)
        res.append(np.linalg.norm(V @ (V.T @ w) - 1.0) / math.sqrt(len(w)))
    assert res[2] < res[1] < res[0]
    assert res[2] < 0.1


def test_radial_weights_grow_with_radius(orc):
    N, K = (32, 32), (64, 64)
    om = data.radial_2d(32, 64)
    w = orc.density_compensation_vvh(om, N, K, 6, 10)
    r = np.linalg.norm(om.astype(np.float64), axis=1)
    inner = w[r < 0.1 * np.pi].mean()
    outer = w[(r > 0.5 * np.pi) & (r < 0.9 * np.pi)].mean()
    assert outer > 3.0 * inner


# ---------------------------------------------------------------- the printed form


def test_printed_step_against_brute_force_nudft(orc):
    """One step of w <- w / (A A^H w) from w = 1 equals the same quotient
    with the exact operator E (E[m, n] = e^{-i omega_m . n}), up to the NUFFT
    approximation error, in both readings."""
    N, K = (8, 8), (16, 16)
    om = np.random.default_rng(11).uniform(-np.pi, np.pi, (60, 2)).astype(np.float32)
    u = nudft_forward(nudft_adjoint(np.ones(60, np.complex128), om, N), om, N)
    assert rel_l2(orc.density_compensation_aah(om, N, K, 6, 1, form="modulus"), 1.0 / np.abs(u)) < 1e-4
    assert rel_l2(orc.density_compensation_aah(om, N, K, 6, 1, form="complex"), 1.0 / u) < 1e-4
    # the product is genuinely complex for this index range (so the reading matters)
    assert np.abs(u.imag).max() > 1e-3 * np.abs(u).max()


def test_printed_modulus_step_is_scale_invariant(orc):
    N, K = (16,), (32,)
    om = np.random.default_rng(1).uniform(-np.pi, np.pi, (50, 1)).astype(np.float32)
    w0 = np.random.default_rng(2).uniform(0.5, 1.5, 50)
    a = orc.density_compensation_aah(om, N, K, 6, 1, w0)
    b = orc.density_compensation_aah(om, N, K, 6, 1, 4.0 * w0)
    assert rel_l2(a, b) < 1e-12


def test_printed_map_does_not_settle_on_radial_sampling(orc):
    """Evenly spaced radial trajectory (32 spokes x 64 readout, image 32^2,
    grid 64^2), float64 throughout.  For the printed map, the fixed-point
    residual r_i = rms(A A^H w_i - 1) after 12 steps is several times the one
    after the first step, and the spread max|w|/min|w| grows by more than an
    order of magnitude (modulus reading; the complex reading jumps around the
    same way).  The V V^H iteration on the same trajectory reduces its own
    residual rms(V V^H w - 1) at every checkpoint (V dense, from scipy)."""
    N, K = (32, 32), (64, 64)
    om = data.radial_2d(32, 64)
    M = om.shape[0]

    def aah_resid(w):
        u = orc.forward(orc.adjoint(np.asarray(w, np.complex128), om, N, K, 6), om, N, K, 6)
        return np.linalg.norm(u - 1.0) / math.sqrt(M)

    for form in ("modulus", "complex"):
        res, spread = [], []
        w = None
        for it in range(12):
            w = orc.density_compensation_aah(om, N, K, 6, 1, w0=w, form=form)
            res.append(aah_resid(w))
            spread.append(np.abs(w).max() / np.abs(w).min())
        print(form, ["%.3g" % r for r in res], "%.3g -> %.3g" % (spread[0], spread[-1]))
        assert max(res[1:]) > 3.0 * res[0]
        assert spread[-1] > 20.0 * spread[0]
        if form == "modulus":
            assert res[-1] > 2.0 * res[0]
    V = _dense_V(om, K, 6)
    vres = []
    for iters in (1, 4, 12):
        w = orc.density_compensation_vvh(om, N, K, 6, iters)
        vres.append(np.linalg.norm(V @ (V.T @ w) - 1.0) / math.sqrt(M))
    assert vres[2] < vres[1] < vres[0]
