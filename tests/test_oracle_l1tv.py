"""Pins of the oracle's L1TV pieces and solvers (paper Section 2.2,
"Iterative NUFFT": image gradient, TV, L1TV-OLS and L1TV-LAD split-Bregman
iterations) against facts that do not come from the oracle:

- the gradient's transpose is its adjoint, and a constant image has zero
  gradient; TV of a 1D step signal is the sum of its jumps (closed form);
- shrink: closed forms for real and complex values, zero threshold is the
  identity, values inside the threshold vanish;
- with a vanishing TV weight, L1TV-OLS reaches the least-squares solution
  (numpy lstsq on the dense NUDFT-like oracle operator);
- on a piecewise-constant phantom with noise, L1TV-OLS lowers both the TV and
  the error against the truth compared with least squares;
- L1TV-LAD with a vanishing TV weight reaches the same least-squares
  solution, and with TV on the noisy phantom it also beats least squares.
"""
import numpy as np
import pytest

from nudft import rel_l2


def _rand_c(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("shape", [(17,), (6, 9), (4, 5, 6)])
def test_gradient_transpose_is_adjoint(orc, shape):
    x, g = _rand_c(shape, 1), _rand_c(shape, 2)
    for a in range(len(shape)):
        lhs = np.vdot(orc.tv_grad(x, a), g)
        rhs = np.vdot(x, orc.tv_grad_t(g, a))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        assert np.abs(orc.tv_grad(np.full(shape, 3 - 2j), a)).max() == 0.0


def test_tv_of_a_step_signal():
    import oracle as orc
    x = np.array([0, 0, 2, 2, 2, -1, -1, 0], dtype=np.complex128)
    # periodic: jumps 2, 3, 1 and the wrap 0 -> 0
    assert orc.tv_norm(x) == pytest.approx(6.0, abs=1e-15)


def test_shrink_closed_forms(orc):
    z = np.array([3.0, -3.0, 0.5, -0.2, 0.0])
    assert np.allclose(orc.shrink(z, 1.0).real, [2.0, -2.0, 0.0, 0.0, 0.0], atol=0)
    c = 3.0 * np.exp(1j * 0.7)
    assert abs(orc.shrink(c, 1.0) - 2.0 * np.exp(1j * 0.7)) < 1e-15
    v = _rand_c((20,), 3)
    assert np.array_equal(orc.shrink(v, 0.0), v)


def _well_posed(M=900, N=(12, 12), seed=5):
    om = np.random.default_rng(seed).uniform(-np.pi, np.pi, (M, len(N))).astype(np.float32)
    return om, N, tuple(2 * n for n in N)


def _dense_A(orc, om, N, K):
    n = int(np.prod(N))
    return np.stack([orc.forward(np.eye(n)[i].reshape(N), om, N, K, 6) for i in range(n)], axis=1)


@pytest.mark.parametrize("lad", [False, True], ids=["ols", "lad"])
def test_vanishing_tv_gives_least_squares(orc, lad):
    om, N, K = _well_posed()
    x_true = _rand_c(N, 6)
    y = orc.forward(x_true, om, N, K, 6) + 0.01 * _rand_c((om.shape[0],), 7)
    x_ls = np.linalg.lstsq(_dense_A(orc, om, N, K), y, rcond=None)[0].reshape(N)
    x = orc.l1tv(y, om, N, K, 6, mu=1.0, lam=1e-7, outer=4, inner=1, cg_iters=30, lad=lad)
    assert rel_l2(x, x_ls) < 1e-6


def _phantom(N):
    x = np.zeros(N, np.complex128)
    x[3:9, 2:7] = 1.0
    x[5:11, 8:11] = 0.5 + 0.3j
    return x


@pytest.mark.parametrize("lad", [False, True], ids=["ols", "lad"])
def test_tv_denoises_piecewise_constant(orc, lad):
    """mu = 3e-3 balances the data term (A^H A ~ M = 700) against the unit TV
    weight of the split formulation; lam = 1 is the splitting penalty."""
    om, N, K = _well_posed(M=700, N=(14, 14), seed=8)
    x_true = _phantom(N)
    y = orc.forward(x_true, om, N, K, 6) + 0.6 * _rand_c((om.shape[0],), 9)
    x_ls = np.linalg.lstsq(_dense_A(orc, om, N, K), y, rcond=None)[0].reshape(N)
    x_tv = orc.l1tv(y, om, N, K, 6, mu=3e-3, lam=1.0, outer=4, inner=4, cg_iters=15, lad=lad)
    assert orc.tv_norm(x_tv) < 0.75 * orc.tv_norm(x_ls)
    assert rel_l2(x_tv, x_true) < 0.5 * rel_l2(x_ls, x_true)
