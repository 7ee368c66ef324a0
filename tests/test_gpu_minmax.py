"""GPU checks of the min-max interpolator (plan option interpolator=1)
against the oracle's direct min-max definition (c = T^-1 r, complex
coefficients, no phase factorisation): forward and adjoint in 1D/2D/3D, on
both gridding paths and both gather paths, with windows that wrap."""
import numpy as np
import pytest

from nudft import nudft_forward, rel_l2
from paper_1710_03197_amd import data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-5


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
    # name, N, J, options, trajectory (wrapping coordinates included)
    ("1d", (64,), 6, {}, lambda: np.random.default_rng(1).uniform(-9, 9, (700, 1)).astype(np.float32)),
    ("2d_mfma", (32, 32), 6, dict(tile=(16, 16)), lambda: np.random.default_rng(2).uniform(-7, 7, (3000, 2)).astype(np.float32)),
    ("2d_valu_direct", (32, 32), 6, dict(tile=(32, 8), grid_mfma=2, interp_direct=1),
     lambda: data.golden_radial_2d(24, 64)),
    ("2d_J5", (24, 20), 5, {}, lambda: np.random.default_rng(3).uniform(-np.pi, np.pi, (2000, 2)).astype(np.float32)),
    ("2d_J8", (32, 32), 8, {}, lambda: np.random.default_rng(4).uniform(-4, 4, (2500, 2)).astype(np.float32)),
    ("3d", (16, 16, 16), 6, {}, lambda: data.koosh_ball_3d(64, 32)),
    ("3d_valu", (12, 12, 12), 6, dict(grid_mfma=2), lambda: np.random.default_rng(5).uniform(-5, 5, (3000, 3)).astype(np.float32)),
]


@pytest.mark.parametrize("name,N,J,opts,traj", CASES, ids=[c[0] for c in CASES])
def test_minmax_matches_oracle(orc, dev, name, N, J, opts, traj):
    from paper_1710_03197_amd import Plan
    om = traj()
    K = tuple(2 * n for n in N)
    x, y = _rand_c(N, 11), _rand_c((om.shape[0],), 12)
    print(f"{name}: N={N} J={J} M={om.shape[0]} options={opts}", flush=True)
    with Plan(_t(om, dev), N, K, J, options=dict(opts, interpolator="minmax")) as p:
        yf = p.forward(_t(x, dev)).cpu().numpy()
        xa = p.adjoint(_t(y, dev)).cpu().numpy()
    ef = rel_l2(yf, orc.minmax_forward(x, om, N, K, J))
    ea = rel_l2(xa, orc.minmax_adjoint(y, om, N, K, J))
    print(f"forward {ef:.2e} adjoint {ea:.2e}", flush=True)
    assert ef < TOL and ea < TOL


def test_minmax_beats_kaiser_bessel_against_nudft(dev):
    from paper_1710_03197_amd import Plan
    N, K = (32, 32), (64, 64)
    om = np.random.default_rng(6).uniform(-np.pi, np.pi, (2000, 2)).astype(np.float32)
    x = _rand_c(N, 7)
    ref = nudft_forward(x, om, N)
    errs = {}
    for interp in ("kb", "minmax"):
        with Plan(_t(om, dev), N, K, 6, options=dict(interpolator=interp)) as p:
            errs[interp] = rel_l2(p.forward(_t(x, dev)).cpu().numpy(), ref)
    print("vs NUDFT:", errs, flush=True)
    assert errs["minmax"] < errs["kb"] < 5e-5


def test_minmax_with_coils_and_batches(orc, dev):
    from paper_1710_03197_amd import Plan
    N, K = (24, 24), (48, 48)
    om = data.golden_radial_2d(16, 48)
    coils = data.coil_maps(N, 3, np.random.default_rng(8)).astype(np.complex64)
    x = _rand_c(N, 9)
    with Plan(_t(om, dev), N, K, 6, coils=_t(coils, dev), options=dict(interpolator=1)) as p:
        ys = p.forward(_t(x, dev)).cpu().numpy()
        xa = p.adjoint(_t(ys, dev)).cpu().numpy()
    for c in range(3):
        assert rel_l2(ys[c], orc.minmax_forward(coils[c] * x, om, N, K, 6)) < TOL
    ref = sum(np.conj(coils[c].astype(np.complex128)) * orc.minmax_adjoint(ys[c], om, N, K, 6) for c in range(3))
    assert rel_l2(xa, ref) < TOL


def test_minmax_rejects_gradients_and_density(dev):
    from paper_1710_03197_amd import NufftError, Plan
    om = data.radial_2d(8, 32)
    with Plan(_t(om, dev), (16, 16), (32, 32), 6, options=dict(interpolator=1)) as p:
        with pytest.raises(NufftError):
            p.grad_points(torch.zeros((16, 16), dtype=torch.complex64, device=dev),
                          torch.zeros(om.shape[0], dtype=torch.complex64, device=dev))
        with pytest.raises(NufftError):
            p.density_compensation(2)
    with pytest.raises(NufftError):
        Plan(_t(om, dev), (16, 16), (32, 32), 6, options=dict(interpolator=2))
    # the window table holds Kaiser-Bessel weights only
    with pytest.raises(NufftError) as ei:
        Plan(_t(om, dev), (16, 16), (32, 32), 6, options=dict(interpolator=1, weight_table=1))
    assert ei.value.code == "NUFFT_ERR_UNSUPPORTED"
