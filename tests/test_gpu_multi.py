"""GPU checks of the multi-problem path (paper Section 2.1 batch mode,
Section 2.2 coils): uneven problems run stage by stage, one kernel launch per
stage and kernel instance over all problems and coils, captured into a HIP
graph per set of buffers.  Against single-plan calls (bitwise: the same
kernels on the same arguments) and against the FP64 oracle, up to the full
size of the 24-problem x 8-coil spiral batch."""
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
    ys2 = mp.forward(xs, ys=[torch.empty_like(y) for y in ys1])  # fresh buffers: new tables and graph
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


def test_multi_mixed_kernel_instances(orc, dev):
    """Problems whose stages need different kernel instances (FFT workgroup
    sizes from K = 24..320, radix 3 and 5, coils or none, pre-sorted samples
    or not, partial sums fused or apart, vector-ALU gridding) share a call;
    each stage still runs as few launches as there are distinct instances."""
    from paper_1710_03197_amd.plan import MultiPlan, Plan
    rng = np.random.default_rng(8)
    spec = [((12, 12), None, None), ((80, 80), 3, None), ((160, 96), None, {"presort": 1}),
            ((48, 48), 2, {"fuse_reduce": 2}), ((64, 64), None, {"grid_mfma": 2, "tile": [16, 8]}),
            ((40, 60), 4, None)]
    probs = []
    for N, C, opt in spec:
        om = data.spiral_2d(int(rng.integers(1500, 6000)), 8, 9)
        probs.append(dict(N=N, K=tuple(2 * n for n in N), om=om, opt=opt,
                          coils=None if C is None else data.coil_maps(N, C, rng).astype(np.complex64),
                          x=data.random_complex_image(N, rng)))
    mp = MultiPlan([dict(om=_t(p["om"], dev), N=p["N"], options=p["opt"],
                         coils=None if p["coils"] is None else _t(p["coils"], dev)) for p in probs], J=6)
    xs = [_t(p["x"], dev) for p in probs]
    ys = mp.forward(xs)
    xa = mp.adjoint(ys)
    torch.cuda.synchronize()
    nf, na = mp.launches()
    print(f"launches per call: forward {nf}, adjoint {na}", flush=True)
    assert 0 < nf < 3 * len(probs) and 0 < na < 4 * len(probs)
    for p, pr in enumerate(probs):
        coils = None if pr["coils"] is None else _t(pr["coils"], dev)
        with Plan(_t(pr["om"], dev), pr["N"], None, 6, coils=coils, options=pr["opt"]) as sp:
            assert np.array_equal(ys[p].cpu().numpy(), sp.forward(xs[p]).cpu().numpy()), p
            assert np.array_equal(xa[p].cpu().numpy(), sp.adjoint(ys[p]).cpu().numpy()), p
        if pr["coils"] is None:
            yo = orc.forward(pr["x"], pr["om"], pr["N"], pr["K"], 6)
            xo = orc.adjoint(ys[p].cpu().numpy(), pr["om"], pr["N"], pr["K"], 6)
        else:
            yo = orc.forward_coils(pr["x"], pr["coils"], pr["om"], pr["N"], pr["K"], 6)
            xo = orc.adjoint_coils(ys[p].cpu().numpy(), pr["coils"], pr["om"], pr["N"], pr["K"], 6)
        assert rel_l2(ys[p].cpu().numpy(), yo) < 1e-5, p
        assert rel_l2(xa[p].cpu().numpy(), xo) < 1e-5, p
    mp.close()


def test_config4_full_size_matches_oracle(orc, dev):
    """The full uneven batch: 24 spiral problems, N in {128..384}^2 (grids
    256..768, radix 3 and 5), M 20k..200k, 8 coils each.  Forward y_i = A(c_i x)
    and coil-combined adjoint of every problem against the FP64 oracle at
    relative L2 <= 1e-5 per problem; the number of launches per call does not
    depend on the number of problems."""
    from paper_1710_03197_amd.plan import MultiPlan
    probs = data.config4()
    print("config 4:", [(p["N"][0], p["om"].shape[0]) for p in probs], flush=True)
    mp = MultiPlan([dict(om=_t(p["om"], dev), N=p["N"], coils=_t(p["coils"], dev)) for p in probs], J=6)
    xs = [_t(p["x"], dev) for p in probs]
    ys = mp.forward(xs)
    xa = mp.adjoint(ys)
    torch.cuda.synchronize()
    nf, na = mp.launches()
    print(f"launches per call: forward {nf}, adjoint {na}", flush=True)
    mp.close()
    ef, ea = [], []
    for p, pr in enumerate(probs):
        y = ys[p].cpu().numpy()
        yo = orc.forward_coils(pr["x"], pr["coils"], pr["om"], pr["N"], pr["K"], 6)
        xo = orc.adjoint_coils(y, pr["coils"], pr["om"], pr["N"], pr["K"], 6)
        ef.append(rel_l2(y, yo))
        ea.append(rel_l2(xa[p].cpu().numpy(), xo))
        # per coil as well: no coil hides behind the others
        ec = max(rel_l2(y[i], yo[i]) for i in range(y.shape[0]))
        assert ec < 1e-5, (p, ec)
    print(f"max rel L2 over problems: forward {max(ef):.2e}, adjoint {max(ea):.2e}", flush=True)
    assert max(ef) < 1e-5 and max(ea) < 1e-5
    # 2D: first pass, strided pass, gather; gridding, inverse pass (summing
    # split tiles), last pass -- one launch each for all 24 problems (a second
    # inverse-pass launch only for problems without split tiles)
    assert nf == 3 and na <= 4


def test_multi_rejects_mixed_dimensions(dev):
    from paper_1710_03197_amd import NufftError
    from paper_1710_03197_amd.plan import MultiPlan
    with pytest.raises(NufftError):
        MultiPlan([dict(om=_t(data.radial_2d(4, 16), dev), N=(8, 8)),
                   dict(om=_t(data.koosh_ball_3d(4, 8), dev), N=(8, 8, 8))])


def test_multi_3d_problems(orc, dev):
    """Three uneven 3D problems (pre-sorted samples, separate partial sums):
    bitwise equal to single plans, oracle parity."""
    from paper_1710_03197_amd.plan import MultiPlan, Plan
    rng = np.random.default_rng(9)
    probs = []
    for N, ns in (((16, 16, 16), 96), ((24, 20, 16), 64), ((12, 12, 12), 40)):
        probs.append(dict(N=N, K=tuple(2 * n for n in N), om=data.koosh_ball_3d(ns, 2 * N[0]),
                          x=data.random_complex_image(N, rng)))
    mp = MultiPlan([dict(om=_t(p["om"], dev), N=p["N"]) for p in probs], J=6)
    xs = [_t(p["x"], dev) for p in probs]
    ys = mp.forward(xs)
    xa = mp.adjoint(ys)
    torch.cuda.synchronize()
    for p, pr in enumerate(probs):
        with Plan(_t(pr["om"], dev), pr["N"], None, 6) as sp:
            assert np.array_equal(ys[p].cpu().numpy(), sp.forward(xs[p]).cpu().numpy()), p
            assert np.array_equal(xa[p].cpu().numpy(), sp.adjoint(ys[p]).cpu().numpy()), p
        assert rel_l2(ys[p].cpu().numpy(), orc.forward(pr["x"], pr["om"], pr["N"], pr["K"], 6)) < 1e-5
        assert rel_l2(xa[p].cpu().numpy(), orc.adjoint(ys[p].cpu().numpy(), pr["om"], pr["N"], pr["K"], 6)) < 1e-5
    mp.close()
