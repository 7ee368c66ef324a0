"""GPU density compensation (nufft_density_compensation) against the
oracle's iterations, and the gridding reconstruction x = A^H (y w)."""
import numpy as np
import pytest

from nudft import rel_l2
from paper_1710_03197_amd import data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


CASES = [("2d radial", (32, 32), lambda: data.radial_2d(24, 64), 10, 6),
         ("1d random", (64,), lambda: np.random.default_rng(3).uniform(-np.pi, np.pi, (300, 1)).astype(np.float32), 5, 6),
         ("3d koosh", (12, 12, 12), lambda: data.koosh_ball_3d(64, 24), 5, 6),
         ("3d koosh J=10", (12, 12, 12), lambda: data.koosh_ball_3d(64, 24), 5, 10)]


@pytest.mark.parametrize("name,N,make_om,iters,J", CASES, ids=[c[0] for c in CASES])
def test_density_compensation_matches_oracle(orc, dev, name, N, make_om, iters, J):
    """Each step divides by V V^H w of the previous iterate; float32 steps
    stay within 1e-4 of the FP64 iterations after `iters` steps."""
    from paper_1710_03197_amd import Plan
    om = make_om()
    K = tuple(2 * n for n in N)
    print(f"{name}: N={N} M={om.shape[0]} iters={iters}", flush=True)
    ref = orc.density_compensation_vvh(om, N, K, J, iters)
    with Plan(_t(om, dev), N, K, J) as p:
        w = p.density_compensation(iters).cpu().numpy()
        e = rel_l2(w, ref)
        print(f"weights rel L2 vs oracle {e:.2e}", flush=True)
        assert e < 1e-4
        # gridding reconstruction with these weights
        y = (np.random.default_rng(5).standard_normal(om.shape[0]) + 0j).astype(np.complex64)
        x = p.adjoint(_t(y, dev) * _t(w, dev)).cpu().numpy()
    assert rel_l2(x, orc.adjoint(y * w.astype(np.float64), om, N, K, J)) < 1e-5


def test_density_compensation_ignores_coils_and_validates(dev):
    from paper_1710_03197_amd import NufftError, Plan
    N, K = (16, 16), (32, 32)
    om = data.radial_2d(12, 32)
    coils = data.coil_maps(N, 3, np.random.default_rng(1)).astype(np.complex64)
    with Plan(_t(om, dev), N, K, 6) as p:
        w1 = p.density_compensation(4).cpu().numpy()
        p.set_coils(_t(coils, dev))
        w2 = p.density_compensation(4).cpu().numpy()
        assert np.array_equal(w1, w2)
        with pytest.raises(NufftError):
            p.density_compensation(-1)


def test_printed_form_matches_oracle(orc, dev):
    """The paper's printed iteration w <- w / |A A^H w| composed from the GPU
    pair, against the oracle's float64 steps.  Two steps: the map amplifies
    rounding (it does not settle on this trajectory), so the comparison stays
    where float32 and float64 iterates are still close."""
    from paper_1710_03197_amd import Plan
    N, K = (32, 32), (64, 64)
    om = data.radial_2d(24, 64)
    ref = orc.density_compensation_aah(om, N, K, 6, 2)
    with Plan(_t(om, dev), N, K, 6) as p:
        w = p.density_compensation(2, form="aah").cpu().numpy()
    e = rel_l2(w, ref)
    print(f"printed form, 2 steps: weights rel L2 vs oracle {e:.2e}", flush=True)
    assert e < 1e-4
