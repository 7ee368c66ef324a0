"""Pins of the oracle's Toeplitz normal operator (paper Section 2.1,
"Self-adjoint NUFFT": A^H A applied with the interpolator out of the loop)
against facts that do not come from the oracle:

- the embedding identity: with the exact point-spread function (brute-force
  NUDFT of the weights on [-N, N)^d) the circulant product equals the exact
  normal operator A^H W A (two NUDFTs) to rounding;
- a closed form: a full Cartesian grid of frequencies 2 pi k / N gives
  A^H A = prod(N) * I;
- Hermitian symmetry of the point-spread function and Hermitian positive
  semi-definiteness of the operator;
- the FFT route of the embedding against the direct sum;
- the NUFFT-made point-spread function against the exact one, and the whole
  Toeplitz operator against the oracle pair A^H (W (A x)), both at the NUFFT
  approximation level.
"""
import numpy as np
import pytest

from nudft import nudft_adjoint, nudft_forward, rel_l2

APPROX_TOL = 5e-5


def _rng(seed):
    return np.random.default_rng(seed)


def _rand_c(shape, seed):
    r = _rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def _rand_om(M, d, seed):
    return _rng(seed).uniform(-np.pi, np.pi, size=(M, d)).astype(np.float32)


def _exact_psf(om, N, w):
    return nudft_adjoint(np.asarray(w, np.complex128), om, tuple(2 * n for n in N))


def _exact_normal(x, om, N, w):
    return nudft_adjoint(np.asarray(w) * nudft_forward(x, om, N), om, N)


@pytest.mark.parametrize("N,M", [((16,), 40), ((8, 6), 70), ((4, 6, 4), 90)])
def test_embedding_identity_with_exact_psf(orc, N, M):
    d = len(N)
    om = _rand_om(M, d, 11 + d)
    w = _rng(5).uniform(0.2, 2.0, M)
    x = _rand_c(N, 7)
    p = _exact_psf(om, N, w)
    ref = _exact_normal(x, om, N, w)
    assert rel_l2(orc.toeplitz_conv(p, x, N), ref) < 1e-12
    assert rel_l2(orc.toeplitz_conv_fft(p, x, N), ref) < 1e-12


def test_cartesian_sampling_gives_scaled_identity(orc):
    N = (8, 8)
    k = np.stack(np.meshgrid(np.arange(-4, 4), np.arange(-4, 4), indexing="ij"), -1).reshape(-1, 2)
    om = (2 * np.pi * k / 8.0).astype(np.float64)
    x = _rand_c(N, 3)
    p = _exact_psf(om, N, np.ones(len(om)))
    assert rel_l2(orc.toeplitz_conv(p, x, N), 64.0 * x) < 1e-12
    # the method's point-spread function (oracle adjoint NUFFT) reaches it to the approximation level
    om32 = om.astype(np.float32)
    out = orc.toeplitz_normal(x, om32, N, (16, 16), 6)
    assert rel_l2(out, 64.0 * x) < APPROX_TOL


def test_psf_hermitian_and_operator_psd(orc):
    N = (6, 8)
    om = _rand_om(80, 2, 21)
    w = _rng(2).uniform(0.5, 1.5, 80)
    p = orc.toeplitz_psf(om, N, (12, 16), 6, w)
    # p[-Delta] = conj(p[Delta]) for Delta in (-N, N): index Delta + N  <->  N - Delta
    P = (12, 16)
    for i0 in range(1, P[0]):
        for i1 in range(1, P[1]):
            assert abs(p[i0, i1] - np.conj(p[P[0] - i0, P[1] - i1])) <= 1e-12 * np.abs(p).max()
    for s in range(4):
        x = _rand_c(N, 30 + s)
        q = np.vdot(x, orc.toeplitz_normal(x, om, N, (12, 16), 6, w))
        assert abs(q.imag) <= 1e-12 * abs(q.real) and q.real > 0


@pytest.mark.parametrize("N,K,M", [((32,), (64,), 300), ((16, 16), (32, 32), 600), ((8, 8, 8), (16, 16, 16), 900)])
def test_method_psf_and_operator_at_approximation_level(orc, N, K, M):
    d = len(N)
    om = _rand_om(M, d, 40 + d)
    w = _rng(9).uniform(0.5, 1.5, M)
    p = orc.toeplitz_psf(om, N, K, 6, w)
    assert rel_l2(p, _exact_psf(om, N, w)) < APPROX_TOL
    x = _rand_c(N, 8)
    t = orc.toeplitz_normal(x, om, N, K, 6, w)
    assert rel_l2(t, _exact_normal(x, om, N, w)) < APPROX_TOL
    pair = orc.adjoint(w * orc.forward(x, om, N, K, 6), om, N, K, 6)
    assert rel_l2(t, pair) < APPROX_TOL
    assert rel_l2(orc.toeplitz_normal(x, om, N, K, 6, w, fft=True), t) < 1e-12


def test_shifted_psf_is_caught(orc):
    """A plausible indexing mistake (PSF off by one cell) fails the identity."""
    N = (8, 6)
    om = _rand_om(50, 2, 3)
    w = np.ones(50)
    x = _rand_c(N, 1)
    p = np.roll(_exact_psf(om, N, w), 1, axis=1)
    assert rel_l2(orc.toeplitz_conv(p, x, N), _exact_normal(x, om, N, w)) > 1e-2
