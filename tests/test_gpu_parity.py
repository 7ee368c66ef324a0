"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded float32 trajectories and complex64 inputs.

Bar: relative L2 error <= 1e-5 (float32 arithmetic against float64), per
stage and for the whole pair; batched and coil modes agree with looped single
calls to 1e-6; the adjoint is bitwise reproducible run to run.
"""
import numpy as np
import pytest

from nudft import rel_l2
from paper_1710_03197_amd import data

pytestmark = pytest.mark.gpu
TOL = 1e-5

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(a, dev, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev) if dtype is None else \
        torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).to(dev)


def _np(t):
    return t.detach().cpu().numpy()


def _rand_c(shape, seed):
    r = np.random.default_rng(seed)
    return (r.standard_normal(shape) + 1j * r.standard_normal(shape)).astype(np.complex64)


def _plan(om, N, K, J, dev, coils=None, options=None):
    from paper_1710_03197_amd import Plan
    return Plan(_t(om, dev), N, K, J, coils=None if coils is None else _t(coils, dev), options=options)


def _bench_options(N, K, J, M):
    """The plan options bench.py times: the shipped tuning cache's entry."""
    from paper_1710_03197_amd.autotune import SHIPPED_CACHE, cached_options
    return cached_options(N, K, J, M, SHIPPED_CACHE)


CASES = [
    # name, N, K, J, trajectory
    ("c1_2d_64", (64, 64), (128, 128), 6, lambda: data.radial_2d(32, 128)),
    ("1d_256", (256,), (512,), 6, lambda: np.random.default_rng(7).uniform(-np.pi, np.pi, (3000, 1)).astype(np.float32)),
    ("3d_16", (16, 16, 16), (32, 32, 32), 6, lambda: data.koosh_ball_3d(64, 32)),
    ("2d_ragged_sigma", (20, 30), (40, 48), 6, lambda: np.random.default_rng(8).uniform(-4, 4, (2500, 2)).astype(np.float32)),
    ("2d_J4_wrap", (32, 48), (64, 96), 4, lambda: np.random.default_rng(9).uniform(-7, 7, (1999, 2)).astype(np.float32)),
    ("2d_J7_odd", (32, 32), (64, 64), 7, lambda: np.random.default_rng(10).uniform(-np.pi, np.pi, (1500, 2)).astype(np.float32)),
    ("3d_ragged", (12, 10, 18), (24, 30, 36), 5, lambda: np.random.default_rng(11).uniform(-np.pi, np.pi, (3000, 3)).astype(np.float32)),
    ("2d_radix35", (192, 160), (384, 320), 6, lambda: data.golden_radial_2d(40, 384)),
    # 12x12x12 tiles: 144 rows of 16 lanes per sample group (not a divisor of 256 lanes)
    ("3d_J10_tile144", (12, 12, 12), (24, 24, 24), 10, lambda: data.koosh_ball_3d(64, 24)),
    ("2d_J12", (24, 24), (48, 48), 12, lambda: data.radial_2d(24, 48)),
]


@pytest.mark.parametrize("name,N,K,J,traj", CASES, ids=[c[0] for c in CASES])
def test_stagewise_and_pair_parity(orc, dev, name, N, K, J, traj):
    om = traj()
    x = _rand_c(N, 1)
    y_in = _rand_c((om.shape[0],), 2)
    print(f"case {name} N={N} K={K} J={J} M={om.shape[0]}", flush=True)
    p = _plan(om, N, K, J, dev)
    # F S
    y_o, g_o, G_o = orc.forward(x, om, N, K, J, stages=True)
    G = p.stage_fs(_t(x, dev))
    assert rel_l2(_np(G), G_o) < TOL
    # V on the oracle's grid (rounded to complex64)
    y_v = p.stage_v(_t(G_o.astype(np.complex64), dev))
    assert rel_l2(_np(y_v), orc.interp(G_o.astype(np.complex64), om, N, K, J)) < TOL
    # V^H alone
    x_o, h_o, H_o = orc.adjoint(y_in, om, N, K, J, stages=True)
    h = p.stage_vh(_t(y_in, dev))
    assert rel_l2(_np(h), h_o) < TOL
    # S^H F^H on the oracle's gridded data
    x_sh = p.stage_shfh(_t(h_o.astype(np.complex64), dev))
    assert rel_l2(_np(x_sh), orc.crop_scale(orc.fftn(h_o.astype(np.complex64), +1), N, K, J)) < TOL
    # whole pair
    y = p.forward(_t(x, dev))
    assert rel_l2(_np(y), y_o) < TOL
    xa = p.adjoint(_t(y_in, dev))
    assert rel_l2(_np(xa), x_o) < TOL
    p.close()


@pytest.mark.parametrize("tuned", [False, True], ids=["defaults", "bench_options"])
def test_config2_full_size(orc, dev, tuned):
    c = data.config2()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    opts = _bench_options(N, K, J, om.shape[0]) if tuned else None
    assert not tuned or opts, "the shipped tuning cache has an entry for this workload"
    p = _plan(om, N, K, J, dev, options=opts)
    y = _np(p.forward(_t(c["x"], dev)))
    y_o = orc.forward(c["x"], om, N, K, J)
    assert rel_l2(y, y_o) < TOL
    yn = (y_o + data.complex_noise(y_o.shape, 1e-3, c["noise_rng"])).astype(np.complex64)
    x = _np(p.adjoint(_t(yn, dev)))
    assert rel_l2(x, orc.adjoint(yn, om, N, K, J)) < TOL
    info = p.info()
    assert info["n_items"] > info["n_bins"]  # the radial centre is split into chunks
    p.close()


@pytest.mark.parametrize("tuned", [False, True], ids=["defaults", "bench_options"])
def test_config3_full_size(orc, dev, tuned):
    c = data.config3()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    opts = _bench_options(N, K, J, om.shape[0]) if tuned else None
    assert not tuned or opts, "the shipped tuning cache has an entry for this workload"
    p = _plan(om, N, K, J, dev, options=opts)
    y = _np(p.forward(_t(c["x"], dev)))
    y_o = orc.forward(c["x"], om, N, K, J)
    assert rel_l2(y, y_o) < TOL
    yin = _rand_c(y.shape, 5)
    x = _np(p.adjoint(_t(yin, dev)))
    assert rel_l2(x, orc.adjoint(yin, om, N, K, J)) < TOL
    p.close()


def test_adjoint_is_deterministic_and_identity_holds(orc, dev):
    """The gridding sums every tile in a fixed order (no atomics), so repeated
    adjoints are bitwise identical; the float32 operator satisfies the adjoint
    identity to float32 rounding."""
    c = data.config1()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    p = _plan(om, N, K, J, dev)
    y = _t(_rand_c((om.shape[0],), 3), dev)
    x1 = _np(p.adjoint(y))
    for _ in range(3):
        assert np.array_equal(_np(p.adjoint(y)).view(np.uint32), x1.view(np.uint32))
    xs = _rand_c(N, 4)
    Ax = _np(p.forward(_t(xs, dev))).astype(np.complex128)
    lhs = np.vdot(_np(y).astype(np.complex128), Ax)
    rhs = np.vdot(x1.astype(np.complex128), xs.astype(np.complex128))
    # float32 operator: the identity holds to float32 rounding
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ax) * np.linalg.norm(_np(y))
    p.close()


def test_empty_trajectory(dev):
    p = _plan(np.zeros((0, 2), np.float32), (16, 16), (32, 32), 6, dev)
    y = p.forward(_t(_rand_c((16, 16), 1), dev))
    assert y.shape == (0,)
    x = _np(p.adjoint(torch.zeros(0, dtype=torch.complex64, device=dev)))
    assert np.all(x == 0)
    p.close()


def test_nonfinite_trajectory_rejected(dev):
    from paper_1710_03197_amd import NufftError, Plan
    om = np.zeros((100, 2), np.float32)
    om[17, 1] = np.nan
    with pytest.raises(NufftError) as ei:
        Plan(_t(om, dev), (16, 16), (32, 32), 6)
    assert ei.value.code == "NUFFT_ERR_NONFINITE"
    good = np.random.default_rng(1).uniform(-3, 3, (100, 2)).astype(np.float32)
    p = Plan(_t(good, dev), (16, 16), (32, 32), 6)
    x = _t(_rand_c((16, 16), 2), dev)
    y0 = _np(p.forward(x))
    with pytest.raises(NufftError):
        p.set_points(_t(om, dev))
    assert np.array_equal(_np(p.forward(x)), y0)  # previous trajectory kept
    p.close()


@pytest.mark.parametrize("opts", [dict(interp_merge=-1), dict(fuse_reduce=3), dict(presort=3), dict(grid_chunk=32),
                                  dict(fft_groups=-1), dict(grid_mfma=4), dict(interpolator=2),
                                  dict(weight_table=2), dict(fft_radix=4), dict(grid_waves=2)],
                         ids=["interp_merge", "fuse_reduce", "presort", "grid_chunk", "fft_groups", "grid_mfma",
                              "interpolator", "weight_table", "fft_radix", "grid_waves"])
def test_out_of_range_options_rejected(dev, opts):
    """Every tuning knob outside its documented range is an argument error."""
    from paper_1710_03197_amd import NufftError, Plan
    om = np.random.default_rng(3).uniform(-3, 3, (200, 2)).astype(np.float32)
    with pytest.raises(NufftError) as ei:
        Plan(_t(om, dev), (16, 16), (32, 32), 6, options=opts)
    assert ei.value.code == "NUFFT_ERR_INVALID_ARG"


def test_batched_equals_looped(dev):
    c = data.config1()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    p = _plan(om, N, K, J, dev)
    xs = np.stack([_rand_c(N, 10 + b) for b in range(3)])
    yb = _np(p.forward_batched(_t(xs, dev)))
    for b in range(3):
        assert rel_l2(yb[b], _np(p.forward(_t(xs[b], dev)))) < 1e-6
    ys = np.stack([_rand_c((om.shape[0],), 20 + b) for b in range(3)])
    xb = _np(p.adjoint_batched(_t(ys, dev)))
    for b in range(3):
        assert rel_l2(xb[b], _np(p.adjoint(_t(ys[b], dev)))) < 1e-6
    p.close()


def test_coil_mode_matches_oracle(orc, dev):
    N, K, J = (48, 40), (96, 80), 6
    om = data.golden_radial_2d(24, 96)
    coils = data.coil_maps(N, 5, np.random.default_rng(3))
    x = _rand_c(N, 4)
    p = _plan(om, N, K, J, dev, coils=coils)
    y = _np(p.forward(_t(x, dev)))
    y_o = orc.forward_coils(x, coils, om, N, K, J)
    assert y.shape == (5, om.shape[0])
    assert rel_l2(y, y_o) < TOL
    ys = np.stack([_rand_c((om.shape[0],), 30 + i) for i in range(5)])
    xa = _np(p.adjoint(_t(ys, dev)))
    assert rel_l2(xa, orc.adjoint_coils(ys, coils, om, N, K, J)) < TOL
    # batched coil mode
    xs = np.stack([x, _rand_c(N, 5)])
    yb = _np(p.forward_batched(_t(xs, dev)))
    assert yb.shape == (2, 5, om.shape[0])
    assert rel_l2(yb[0], y) < 1e-6
    p.close()


def test_many_coils_multiple_rounds(orc, dev):
    """More coils than one LDS tile holds: the last pass combines coils over
    several rounds."""
    N, K, J = (64, 64), (512, 512), 6
    om = data.golden_radial_2d(8, 256)
    coils = data.coil_maps(N, 20, np.random.default_rng(6))
    p = _plan(om, N, K, J, dev, coils=coils)
    ys = np.stack([_rand_c((om.shape[0],), 40 + i) for i in range(20)])
    xa = _np(p.adjoint(_t(ys, dev)))
    assert rel_l2(xa, orc.adjoint_coils(ys, coils, om, N, K, J)) < TOL
    p.close()


def test_trajectory_gradient_matches_oracle(orc, dev):
    N, K, J = (32, 24), (64, 48), 6
    om = data.perturb(data.golden_radial_2d(16, 64), K, np.random.default_rng(2))
    coils = data.coil_maps(N, 3, np.random.default_rng(4))
    x = _rand_c(N, 5)
    gy = np.stack([_rand_c((om.shape[0],), 50 + i) for i in range(3)])
    p = _plan(om, N, K, J, dev, coils=coils)
    g = _np(p.grad_points(_t(x, dev), _t(gy, dev)))
    ref = np.zeros((om.shape[0], 2))
    for i in range(3):
        G = orc.forward_grid(coils[i].astype(np.complex128) * x, N, K, J)
        orc.grad_points(G, gy[i], om, N, K, J, out=ref)
    assert rel_l2(g, ref) < 1e-4
    p.close()


def test_trajectory_gradient_3d(orc, dev):
    N, K, J = (12, 16, 10), (24, 32, 20), 6
    om = np.random.default_rng(12).uniform(-np.pi, np.pi, (800, 3)).astype(np.float32)
    x = _rand_c(N, 6)
    gy = _rand_c((800,), 7)
    p = _plan(om, N, K, J, dev)
    g = _np(p.grad_points(_t(x, dev), _t(gy, dev)))
    ref = orc.grad_points(orc.forward_grid(x, N, K, J), gy, om, N, K, J)
    assert rel_l2(g, ref) < 1e-4
    p.close()


def test_pair_captured_in_a_graph_replays_exactly(dev):
    """forward + adjoint launch only kernels on the caller's stream (no
    allocation, no memset once the workspace exists), so torch can capture
    them; every replay, with eager work in between, equals the eager result."""
    from paper_1710_03197_amd import Plan
    c = data.config1()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    p = Plan(_t(om, dev), N, K, J)
    x = _t(c["x"], dev)
    y = torch.empty(om.shape[0], dtype=torch.complex64, device=dev)
    xa = torch.empty(N, dtype=torch.complex64, device=dev)
    p.forward(x, out=y)
    p.adjoint(y, out=xa)
    torch.cuda.synchronize()
    y_ref, x_ref = y.cpu().numpy(), xa.cpu().numpy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.forward(x, out=y)
        p.adjoint(y, out=xa)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.forward(x, out=y)
        p.adjoint(y, out=xa)
    for k in range(3):
        y.zero_()
        xa.zero_()
        p.forward(torch.zeros_like(x))  # unrelated eager work on the same plan between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), y_ref), k
        assert np.array_equal(xa.cpu().numpy(), x_ref), k
    p.close()


OPTION_CASES = [
    ((64, 64), dict(tile=(16, 16), grid_chunk=256, fft_groups=256)),
    ((64, 64), dict(tile=(64, 8), grid_chunk=2048, fft_groups=4096, interp_direct=1)),
    ((64, 64), dict(tile=(16, 32), grid_chunk=64, presort=1, fuse_reduce=1)),
    ((16, 16, 16), dict(tile=(4, 4, 16), grid_chunk=2048, fft_groups=2048)),
    ((16, 16, 16), dict(tile=(16, 8, 8), grid_chunk=128, interp_direct=1, presort=2, fuse_reduce=2)),
    ((16, 16, 16), dict(tile=(8, 8, 8), grid_chunk=64, presort=2, fuse_reduce=1)),
    ((64,), dict(tile=(16,), grid_chunk=64, presort=1, fuse_reduce=1)),
    ((64, 64), dict(tile=(16, 16), grid_mfma=2)),
    ((64, 64), dict(tile=(32, 16), grid_chunk=128, grid_mfma=1, presort=1)),
    ((64, 64), dict(tile=(16, 16), grid_chunk=64, grid_mfma=1, fuse_reduce=2)),
    ((8, 8), dict(tile=(16, 16), grid_mfma=1)),                  # one tile per axis: wrapped windows
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_mfma=1, presort=2)),
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_mfma=2)),
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_chunk=64, grid_mfma=1, fuse_reduce=2)),
    ((8, 8, 8), dict(tile=(8, 8, 16), grid_mfma=1)),              # last axis one tile
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_mfma=3)),            # row tiles where blocks apply
    ((32, 32, 32), dict(tile=(16, 16, 16), grid_chunk=128)),       # row-tile kernel does not fit: vector ALUs
    ((32, 32, 32), dict(tile=(16, 8, 16), grid_chunk=256, presort=2)),
    ((32, 32, 32), dict(tile=(8, 16, 16), fuse_reduce=1)),
    ((4, 4, 8), dict(tile=(8, 8, 16))),                            # every axis one tile: wrapped windows
    ((64, 64), dict(tile=(16, 16), interp_merge=4)),             # gather items over runs of tiles
    ((64, 64), dict(tile=(16, 16), weight_table=1)),             # windows from the plan's table
    ((64, 64), dict(tile=(32, 16), weight_table=1, interp_merge=2, presort=1)),
    ((16, 16, 16), dict(tile=(8, 8, 16), weight_table=1)),
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_mfma=3, weight_table=1)),
    ((4, 4, 8), dict(tile=(8, 8, 16), weight_table=1)),
    ((64,), dict(tile=(16,), weight_table=1)),
    ((96, 80), dict(fft_radix=1)),                               # radix schedules, K = 192 x 160
    ((96, 80), dict(fft_radix=2)),
    ((96, 80), dict(fft_radix=3)),
    ((64, 64), dict(fft_radix=1, tile=(16, 16))),
    ((16, 16, 16), dict(fft_radix=3, tile=(8, 8, 16))),
    ((120,), dict(fft_radix=2, tile=(16,))),
    ((16, 16, 16), dict(tile=(8, 8, 8), interp_merge=3)),
    ((64,), dict(tile=(16,), interp_merge=5)),
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_waves=1)),            # block gridding, one wavefront per item
    ((32, 32, 32), dict(tile=(16, 8, 16), grid_waves=1, grid_chunk=64, presort=2)),
    ((32, 32, 32), dict(tile=(8, 16, 16), grid_waves=1, weight_table=1, fuse_reduce=1)),
    ((4, 4, 8), dict(tile=(8, 8, 16), grid_waves=1)),               # wrapped windows
    ((16, 16, 16), dict(tile=(8, 8, 16), grid_waves=1, grid_mfma=2)),  # ignored off the block kernel
    ((96, 80), dict(tile=(16, 10), grid_chunk=64)),               # split tiles summed cell by cell (rows of 10)
    ((96, 80), dict(tile=(16, 10), grid_chunk=64, interp_merge=3)),
]


@pytest.mark.parametrize("N,opts", OPTION_CASES, ids=[str(i) for i in range(len(OPTION_CASES))])
def test_tuning_options_keep_parity(orc, dev, N, opts):
    """Every knob the autotuner turns gives the same operator."""
    from paper_1710_03197_amd import Plan
    K = tuple(2 * n for n in N)
    om = {1: lambda: data.perturb(np.linspace(-np.pi, np.pi, 3000, endpoint=False)[:, None].astype(np.float32),
                                  (128,), np.random.default_rng(9)),
          2: lambda: data.radial_2d(48, 128), 3: lambda: data.koosh_ball_3d(96, 32)}[len(N)]()
    x = _rand_c(N, 7)
    yin = _rand_c((om.shape[0],), 8)
    print(f"N={N} options={opts}", flush=True)
    with Plan(_t(om, dev), N, K, 6, options=opts) as p:
        assert rel_l2(_np(p.forward(_t(x, dev))), orc.forward(x, om, N, K, 6)) < TOL
        assert rel_l2(_np(p.adjoint(_t(yin, dev))), orc.adjoint(yin, om, N, K, 6)) < TOL
        assert rel_l2(_np(p.stage_vh(_t(yin, dev))), orc.grid(yin, om, N, K, 6)) < TOL


@pytest.mark.parametrize("N,opts", [((64, 64), dict(tile=(16, 16), grid_chunk=64)),
                                    ((64, 64), dict(tile=(16, 32), grid_chunk=64, grid_mfma=2)),
                                    ((16, 16, 16), dict(tile=(8, 8, 16), grid_chunk=64))],
                         ids=["2d_mfma", "2d_valu", "3d_mfma"])
def test_split_tile_sums_agree_bitwise(dev, N, opts):
    """The partial tiles of split gridding tiles are summed either by the first
    inverse FFT pass or by a kernel of their own; both add the same numbers in
    the same chunk order, so the adjoints agree bit for bit, single and
    batched (per-grid partial slots)."""
    from paper_1710_03197_amd import Plan
    K = tuple(2 * n for n in N)
    om = data.radial_2d(48, 128) if len(N) == 2 else data.koosh_ball_3d(96, 32)
    y = _t(np.stack([_rand_c((om.shape[0],), 80 + b) for b in range(3)]), dev)
    out = {}
    for mode in (1, 2):
        with Plan(_t(om, dev), N, K, 6, options=dict(opts, fuse_reduce=mode)) as p:
            info = p.info()
            assert info["n_items"] > int(np.prod([k // t for k, t in zip(K, info["tile"])]))  # some tiles split
            out[mode] = (_np(p.adjoint(y[0])), _np(p.adjoint_batched(y)))
    assert np.array_equal(out[1][0].view(np.uint32), out[2][0].view(np.uint32))
    assert np.array_equal(out[1][1].view(np.uint32), out[2][1].view(np.uint32))
    assert np.array_equal(out[2][1][0].view(np.uint32), out[2][0].view(np.uint32))


@pytest.mark.parametrize("N,K", [((16, 16), (16, 32)), ((8, 12, 8), (8, 24, 16))])
def test_axis_without_oversampling_matches_oracle(orc, dev, N, K):
    """K_a = N_a on a leading axis: the strided FFT passes must still centre
    the image on that axis (no zero rows to skip there; a missing shift gives
    O(1) errors).  Without oversampling the deapodization 1/Phi(n/K) spans a
    factor ~3500 across the image (J = 6, sigma = 1), which magnifies the
    float32 rounding of the path, so the bar here is 5e-4."""
    from paper_1710_03197_amd import Plan
    d = len(N)
    om = np.random.default_rng(61).uniform(-np.pi, np.pi, (1500, d)).astype(np.float32)
    x = _rand_c(N, 62)
    yin = _rand_c((1500,), 63)
    with Plan(_t(om, dev), N, K, 6) as p:
        assert rel_l2(_np(p.forward(_t(x, dev))), orc.forward(x, om, N, K, 6)) < 5e-4
        assert rel_l2(_np(p.adjoint(_t(yin, dev))), orc.adjoint(yin, om, N, K, 6)) < 5e-4


@pytest.mark.parametrize("N,traj", [((64,), lambda: np.random.default_rng(21).uniform(-np.pi, np.pi, (900, 1))),
                                    ((48, 40), lambda: data.radial_2d(32, 96)),
                                    ((16, 16, 16), lambda: data.koosh_ball_3d(64, 32))],
                         ids=["1d", "2d", "3d"])
def test_gather_reads_unaligned_grids(orc, dev, N, traj):
    """The gather stages its region by 16-byte pairs of cells when the grid is
    16-byte aligned and element by element otherwise: a grid 8 bytes off a
    16-byte boundary gives the same bits as an aligned copy."""
    from paper_1710_03197_amd import Plan
    om = traj().astype(np.float32)
    K = tuple(2 * n for n in N)
    G = _rand_c(K, 22)
    with Plan(_t(om, dev), N, K, 6) as p:
        aligned = _t(G, dev)
        buf = torch.empty(int(np.prod(K)) + 1, dtype=torch.complex64, device=dev)
        shifted = buf[1:].view(K)
        shifted.copy_(aligned)
        assert aligned.data_ptr() % 16 == 0 and shifted.data_ptr() % 16 == 8
        y_a = _np(p.stage_v(aligned))
        y_s = _np(p.stage_v(shifted))
    assert np.array_equal(y_a.view(np.uint32), y_s.view(np.uint32))
    assert rel_l2(y_a, orc.interp(G, om, N, K, 6)) < TOL
