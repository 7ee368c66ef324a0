"""GPU checks of the Toeplitz normal operator (nufft_toeplitz_*) against the
oracle's Toeplitz operator (point-spread function from the FP64 adjoint on
the doubled grid, direct circulant sum), and against the pair A^H W A."""
import numpy as np
import pytest

from nudft import rel_l2
from paper_1710_03197_amd import data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-5          # float32 path vs the FP64 oracle of the same algorithm
APPROX_TOL = 5e-5   # Toeplitz vs the pair: two different approximations of A^H W A


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _rand_c(shape, seed):
    r = np.random.default_rng(seed)
    return (r.standard_normal(shape) + 1j * r.standard_normal(shape)).astype(np.complex64)


CASES = [
    ((48,), 500, False),
    ((48,), 500, True),
    ((24, 20), 1500, False),
    ((32, 32), 3000, True),
    ((12, 10, 8), 2500, True),
]


@pytest.mark.parametrize("N,M,weighted", CASES, ids=[f"{len(c[0])}d-{c[0][0]}-{'w' if c[2] else '1'}" for c in CASES])
def test_toeplitz_matches_oracle(orc, dev, N, M, weighted):
    from paper_1710_03197_amd import Plan
    d = len(N)
    K = tuple(2 * n for n in N)
    om = np.random.default_rng(100 + d).uniform(-np.pi, np.pi, (M, d)).astype(np.float32)
    w = np.random.default_rng(7).uniform(0.3, 2.0, M).astype(np.float32) if weighted else None
    x = _rand_c(N, 3)
    print(f"N={N} M={M} weighted={weighted}", flush=True)
    ref = orc.toeplitz_normal(x, om, N, K, 6, None if w is None else w.astype(np.float64))
    with Plan(_t(om, dev), N, K, 6) as p:
        with p.toeplitz(None if w is None else _t(w, dev)) as T:
            out = T(_t(x, dev)).cpu().numpy()
            assert rel_l2(out, ref) < TOL
            # the pair gives the same operator to the approximation level
            yy = p.forward(_t(x, dev))
            if w is not None:
                yy = yy * _t(w, dev)
            pair = p.adjoint(yy).cpu().numpy()
            assert rel_l2(out, pair) < APPROX_TOL
            # batched: B images in one call equal B single calls
            xb = np.stack([_rand_c(N, 20 + b) for b in range(3)])
            ob = T(_t(xb, dev)).cpu().numpy()
            for b in range(3):
                assert np.array_equal(ob[b], T(_t(xb[b], dev)).cpu().numpy())


def test_toeplitz_with_coils(orc, dev):
    from paper_1710_03197_amd import Plan
    N, K, M = (32, 32), (64, 64), 2500
    om = data.golden_radial_2d(10, 250)
    coils = data.coil_maps(N, 4, np.random.default_rng(2)).astype(np.complex64)
    x = _rand_c(N, 5)
    p_ref = orc.toeplitz_psf(om, N, K, 6)
    ref = sum(np.conj(c.astype(np.complex128)) * orc.toeplitz_conv(p_ref, c * x, N) for c in coils)
    with Plan(_t(om, dev), N, K, 6, coils=_t(coils, dev)) as p:
        with p.toeplitz() as T:
            out = T(_t(x, dev)).cpu().numpy()
    assert rel_l2(out, ref) < TOL


def test_toeplitz_config2_full_size(orc, dev):
    """2D 256^2 on the 512^2 grid, 131072 golden-angle samples: against the
    oracle's FFT route of the same operator."""
    from paper_1710_03197_amd import Plan
    c = data.config2()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    x = c["x"].astype(np.complex64)
    ref = orc.toeplitz_normal(x, om, N, K, J, fft=True)
    with Plan(_t(om, dev), N, K, J) as p:
        with p.toeplitz() as T:
            out = T(_t(x, dev)).cpu().numpy()
    e = rel_l2(out, ref)
    print(f"config 2 Toeplitz rel L2 vs oracle {e:.2e}", flush=True)
    assert e < TOL


def test_toeplitz_cg_matches_oracle(orc, dev):
    """10 CG iterations on A^H A x = A^H y with the Toeplitz operator against
    the same iterations with the oracle's Toeplitz operator, on a
    well-conditioned problem (8 samples per image pixel, uniform random):
    there the float64 iterate moves by ~1.5e-6 under 1e-6 relative operator
    noise, so float32 arithmetic must land within 1e-4.  (An undersampled
    radial problem such as config 1 moves by ~1e-2 under the same noise.)"""
    from paper_1710_03197_amd import Plan
    from paper_1710_03197_amd.solvers import cg_normal
    N, K, J = (32, 32), (64, 64), 6
    om = np.random.default_rng(5).uniform(-np.pi, np.pi, (8192, 2)).astype(np.float32)
    x_true = _rand_c(N, 6)
    y = orc.forward(x_true, om, N, K, J).astype(np.complex64)
    psf = orc.toeplitz_psf(om, N, K, J)
    x_orc, _ = orc.cg(lambda v: orc.toeplitz_conv(psf, v, N), orc.adjoint(y, om, N, K, J), 10)
    with Plan(_t(om, dev), N, K, J) as p:
        with p.toeplitz() as T:
            x_gpu = cg_normal(p, _t(y, dev), iters=10, normal=T).cpu().numpy()
    e = rel_l2(x_gpu, x_orc)
    print(f"Toeplitz CG 10 iterations: GPU vs oracle rel L2 {e:.2e}", flush=True)
    assert e < 1e-4


def test_toeplitz_rejects_bad_input(dev):
    from paper_1710_03197_amd import NufftError, Plan
    om = data.radial_2d(4, 16)
    with Plan(_t(om, dev), (8, 8), (16, 16), 6) as p:
        w = torch.full((om.shape[0],), float("nan"), device=dev)
        with pytest.raises(NufftError):
            p.toeplitz(w)


def test_toeplitz_empty_trajectory_and_growing_batches(dev):
    """No samples: the operator is zero.  A larger batch after a smaller one
    grows the workspace and gives the same per-image results."""
    from paper_1710_03197_amd import Plan
    N, K = (16, 12), (32, 24)
    with Plan(torch.empty((0, 2), dtype=torch.float32, device=dev), N, K, 6) as p:
        with p.toeplitz() as T:
            out = T(_t(_rand_c(N, 1), dev)).cpu().numpy()
        assert np.abs(out).max() == 0.0
        assert p.density_compensation(3).numel() == 0
    om = np.random.default_rng(2).uniform(-np.pi, np.pi, (700, 2)).astype(np.float32)
    with Plan(_t(om, dev), N, K, 6) as p:
        with p.toeplitz() as T:
            x1 = _rand_c((1,) + N, 3)
            o1 = T(_t(x1, dev)).cpu().numpy()
            x5 = np.concatenate([x1, np.stack([_rand_c(N, 10 + b) for b in range(4)])])
            o5 = T(_t(x5, dev)).cpu().numpy()
    assert np.array_equal(o1[0], o5[0])
