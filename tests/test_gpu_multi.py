"""GPU checks of the multi-problem path (uneven problems with coils, captured
into one HIP graph and replayed) against single-plan calls and the oracle."""
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


def test_multi_matches_single_plans_and_oracle(orc, dev):
    from paper_1710_03197_amd.plan import MultiPlan, Plan
    probs = data.config4(seed=41, n_problems=5, n_coils=3, sizes=(32, 48, 64), m_range=(2000, 9000))
    print("problems:", [(p["N"], p["om"].shape[0]) for p in probs], flush=True)
    mp = MultiPlan([dict(om=_t(p["om"], dev), N=p["N"], coils=_t(p["coils"], dev)) for p in probs], J=6)
    xs = [_t(p["x"], dev) for p in probs]
    ys1 = mp.forward(xs)
    ys2 = mp.forward(xs, ys=[torch.empty_like(y) for y in ys1])  # fresh buffers: a second capture
    ys3 = mp.forward(xs, ys=ys2)                                  # same buffers: a replay
    torch.cuda.synchronize()
    for p, pr in enumerate(probs):
        with Plan(_t(pr["om"], dev), pr["N"], None, 6, coils=_t(pr["coils"], dev)) as sp:
            ref = sp.forward(xs[p]).cpu().numpy()
            assert np.array_equal(ys1[p].cpu().numpy(), ref)
            assert np.array_equal(ys3[p].cpu().numpy(), ref)
            xa = mp.adjoint(ys1)[p].cpu().numpy()
            assert np.array_equal(xa, sp.adjoint(ys1[p]).cpu().numpy())
        yo = orc.forward_coils(pr["x"], pr["coils"], pr["om"], pr["N"], pr["K"], 6)
        assert rel_l2(ys1[p].cpu().numpy(), yo) < 1e-5
    mp.close()


def test_multi_rejects_mixed_dimensions(dev):
    from paper_1710_03197_amd import NufftError
    from paper_1710_03197_amd.plan import MultiPlan
    with pytest.raises(NufftError):
        MultiPlan([dict(om=_t(data.radial_2d(4, 16), dev), N=(8, 8)),
                   dict(om=_t(data.koosh_ball_3d(4, 8), dev), N=(8, 8, 8))])
