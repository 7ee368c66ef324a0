"""Pins of the oracle's sampling-density compensation (paper Section 2.2,
"Density compensation and gridding": w <- w / A A^H w, after Pipe and Menon;
modulus reading) against facts that do not come from the oracle:

- a full Cartesian set of frequencies 2 pi k / N gives A A^H = prod(N) I, so
  the weights are 1 / prod(N) after one step and stay there;
- one step against the brute-force NUDFT;
- scale invariance of a step (w -> c w gives the same next iterate);
- on a radial trajectory the weights grow with the distance from the centre
  (the density of radial samples falls as 1/|k|).
"""
import numpy as np

from nudft import nudft_adjoint, nudft_forward, rel_l2
from paper_1710_03197_amd import data

APPROX_TOL = 5e-5


def test_cartesian_weights_are_uniform(orc):
    N = (8, 8)
    k = np.stack(np.meshgrid(np.arange(-4, 4), np.arange(-4, 4), indexing="ij"), -1).reshape(-1, 2)
    om = (2 * np.pi * k / 8.0).astype(np.float32)
    for iters in (1, 3):
        w = orc.density_compensation(om, N, (16, 16), 6, iters)
        assert rel_l2(w, np.full(len(om), 1.0 / 64)) < APPROX_TOL


def test_one_step_against_brute_force(orc):
    N = (6, 8)
    om = np.random.default_rng(4).uniform(-np.pi, np.pi, (120, 2)).astype(np.float32)
    ref = 1.0 / np.abs(nudft_forward(nudft_adjoint(np.ones(120), om, N), om, N))
    assert rel_l2(orc.density_compensation(om, N, (12, 16), 6, 1), ref) < APPROX_TOL


def test_step_is_scale_invariant(orc):
    N, K = (16,), (32,)
    om = np.random.default_rng(1).uniform(-np.pi, np.pi, (50, 1)).astype(np.float32)
    w0 = np.random.default_rng(2).uniform(0.5, 1.5, 50)
    a = orc.density_compensation(om, N, K, 6, 1, w0)
    b = orc.density_compensation(om, N, K, 6, 1, 7.5 * w0)
    assert rel_l2(a, b) < 1e-12


def test_radial_weights_grow_with_radius(orc):
    N, K = (32, 32), (64, 64)
    om = data.radial_2d(32, 64)
    w = orc.density_compensation(om, N, K, 6, 10)
    r = np.linalg.norm(om.astype(np.float64), axis=1)
    inner = w[r < 0.1 * np.pi].mean()
    outer = w[(r > 0.5 * np.pi) & (r < 0.9 * np.pi)].mean()
    assert outer > 3.0 * inner
