"""GPU checks of the L1TV pieces (nufft_tv_*, nufft_bregman_shrink) against
the oracle's formulas, and of the L1TV-OLS / L1TV-LAD solvers against the
oracle's iterations."""
import numpy as np
import pytest

from nudft import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("shape", [(37,), (9, 14), (5, 7, 6)])
def test_tv_kernels_match_oracle(orc, dev, shape):
    from paper_1710_03197_amd import solvers
    d = len(shape)
    x, b0 = _rand_c(shape, 1), _rand_c((d,) + shape, 2)
    dd0, ahy = _rand_c((d,) + shape, 3), _rand_c(shape, 4)
    t, mu, lam = 0.7, 0.3, 1.9
    # shrink + Bregman update
    dd, bb = torch.empty((d,) + shape, dtype=torch.complex64, device=dev), _t(b0, dev)
    solvers.tv_shrink(_t(x, dev), dd, bb, t)
    for a in range(d):
        z = orc.tv_grad(x.astype(np.complex128), a) + b0[a]
        assert rel_l2(dd[a].cpu().numpy(), orc.shrink(z, t)) < 1e-6
        assert rel_l2(bb[a].cpu().numpy(), z - orc.shrink(z, t)) < 1e-6
    # right-hand side (OLS and LAD forms)
    out = torch.empty(shape, dtype=torch.complex64, device=dev)
    solvers.tv_rhs(mu, _t(ahy, dev), lam, _t(dd0, dev), _t(b0, dev), out)
    ref = mu * ahy.astype(np.complex128) + lam * sum(orc.tv_grad_t(dd0[a] - b0[a], a) for a in range(d))
    assert rel_l2(out.cpu().numpy(), ref) < 1e-6
    df, bf = _rand_c(shape, 5), _rand_c(shape, 6)
    solvers.tv_rhs(mu, _t(ahy, dev), lam, _t(dd0, dev), _t(b0, dev), out, _t(df, dev), _t(bf, dev))
    ref = mu * (ahy + df - bf).astype(np.complex128) + lam * sum(orc.tv_grad_t(dd0[a] - b0[a], a) for a in range(d))
    assert rel_l2(out.cpu().numpy(), ref) < 1e-6
    # system matrix K applied to x (A^H A x supplied)
    solvers.tv_normal(mu, _t(ahy, dev), lam, _t(x, dev), out)
    ref = mu * ahy.astype(np.complex128) + lam * sum(orc.tv_grad_t(orc.tv_grad(x.astype(np.complex128), a), a)
                                                     for a in range(d))
    assert rel_l2(out.cpu().numpy(), ref) < 1e-6
    # elementwise Bregman shrink
    r = _rand_c(shape, 7)
    dv, bv = torch.empty(shape, dtype=torch.complex64, device=dev), _t(bf, dev)
    solvers.bregman_shrink(_t(r, dev), dv, bv, t)
    z = r.astype(np.complex128) + bf
    assert rel_l2(dv.cpu().numpy(), orc.shrink(z, t)) < 1e-6
    assert rel_l2(bv.cpu().numpy(), z - orc.shrink(z, t)) < 1e-6


def _phantom(N):
    x = np.zeros(N, np.complex128)
    x[3:9, 2:7] = 1.0
    x[5:11, 8:11] = 0.5 + 0.3j
    return x


@pytest.mark.parametrize("lad", [False, True], ids=["ols", "lad"])
@pytest.mark.parametrize("op", ["pair", "toeplitz"])
def test_l1tv_matches_oracle(orc, dev, lad, op):
    """The iterations (4 outer x 4 inner, 15 CG steps each) on the noisy
    phantom of the oracle pins, against the oracle's FP64 iterations."""
    from paper_1710_03197_amd import Plan
    from paper_1710_03197_amd.solvers import l1tv
    N, K = (16, 16), (32, 32)   # 2-3-5 smooth grid sizes (the oracle pins use 14 x 14)
    om = np.random.default_rng(8).uniform(-np.pi, np.pi, (900, 2)).astype(np.float32)
    y = (orc.forward(_phantom(N), om, N, K, 6) + 0.6 * _rand_c((900,), 9)).astype(np.complex64)
    ref = orc.l1tv(y, om, N, K, 6, mu=3e-3, lam=1.0, outer=4, inner=4, cg_iters=15, lad=lad)
    with Plan(_t(om, dev), N, K, 6) as p:
        T = p.toeplitz() if op == "toeplitz" else None
        x = l1tv(p, _t(y, dev), mu=3e-3, lam=1.0, outer=4, inner=4, cg_iters=15, lad=lad, normal=T).cpu().numpy()
        if T is not None:
            T.close()
    e = rel_l2(x, ref)
    print(f"L1TV {'LAD' if lad else 'OLS'} ({op}) GPU vs oracle rel L2 {e:.2e}; "
          f"error vs truth {rel_l2(x, _phantom(N)):.3e} (oracle {rel_l2(ref, _phantom(N)):.3e})", flush=True)
    assert e < (1e-4 if op == "pair" else 1e-3)
