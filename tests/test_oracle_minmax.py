"""Pins of the oracle's min-max interpolator (the paper's default kernel,
Section 2.1 "Interpolation", after Fessler and Sutton) against facts that do
not come from the oracle:

- least-squares optimality, the defining property: for each sample the
  coefficients minimise ||e^{-i omega n} - s_n sum_j c_j e^{-i gamma (k0+j) n}||
  over n, so random perturbations of c only increase that error;
- accuracy against the brute-force NUDFT, better than the Kaiser-Bessel
  interpolator at the same J and oversampling;
- the adjoint is the conjugate transpose;
- the factorisation the GPU path uses: with the half-integer scaling centres,
  c_j e^{-i gamma t_j / 2} is real (t_j = u - k0 - j).
"""
import numpy as np
import pytest

from nudft import nudft_adjoint, nudft_forward, rel_l2


def _rand_c(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def test_coefficients_are_least_squares_optimal(orc):
    N, K, J = 24, 48, 6
    om = np.random.default_rng(1).uniform(-np.pi, np.pi, 40)
    k0, c = orc.minmax_coefs(om, N, K, J)
    s = orc.minmax_scaling(N, K, J)
    n = np.arange(N) - N // 2
    g = 2 * np.pi / K
    rng = np.random.default_rng(2)
    for m in range(len(om)):
        B = s[:, None] * np.exp(-1j * g * (k0[m] + np.arange(J))[None, :] * n[:, None])
        a = np.exp(-1j * om[m] * n)
        e0 = np.linalg.norm(a - B @ c[m])
        # the normal equations hold and no perturbation does better
        assert np.abs(B.conj().T @ (a - B @ c[m])).max() <= 1e-9 * np.abs(B.conj().T @ a).max()
        for _ in range(5):
            dlt = 1e-3 * np.abs(c[m]).max() * (rng.standard_normal(J) + 1j * rng.standard_normal(J))
            assert np.linalg.norm(a - B @ (c[m] + dlt)) > e0


@pytest.mark.parametrize("N,K,M", [((32,), (64,), 400), ((16, 12), (32, 24), 600), ((8, 8, 8), (16, 16, 16), 700)])
def test_accuracy_against_nudft(orc, N, K, M):
    d = len(N)
    om = np.random.default_rng(3 + d).uniform(-np.pi, np.pi, (M, d)).astype(np.float32)
    x, y = _rand_c(N, 5), _rand_c((M,), 6)
    e_mm = rel_l2(orc.minmax_forward(x, om, N, K, 6), nudft_forward(x, om, N))
    e_kb = rel_l2(orc.forward(x, om, N, K, 6), nudft_forward(x, om, N))
    assert e_mm < 5e-5 and e_mm < e_kb
    assert rel_l2(orc.minmax_adjoint(y, om, N, K, 6), nudft_adjoint(y, om, N)) < 5e-5


def test_adjoint_is_conjugate_transpose(orc):
    N, K = (10, 12), (20, 24)
    om = np.random.default_rng(7).uniform(-5, 5, (300, 2)).astype(np.float32)
    x, y = _rand_c(N, 8), _rand_c((300,), 9)
    lhs = np.vdot(orc.minmax_forward(x, om, N, K, 6), y)
    rhs = np.vdot(x, orc.minmax_adjoint(y, om, N, K, 6))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("J", [4, 6, 7])
def test_half_sample_phase_factorisation(orc, J):
    N, K = 32, 64
    om = np.random.default_rng(J).uniform(-9, 9, 200)      # includes windows that wrap
    k0, c = orc.minmax_coefs(om, N, K, J)
    u = om * K / (2 * np.pi)
    t = u[:, None] - k0[:, None] - np.arange(J)[None, :]
    cr = c * np.exp(-1j * (np.pi / K) * t)
    assert np.abs(cr.imag).max() <= 1e-12 * np.abs(cr).max()
