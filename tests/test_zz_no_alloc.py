"""The allocation-free density compensation (nufft_density_compensation_noalloc,
which takes its sample buffers from a static device array) against the
allocating entry point nufft_density_compensation on the same plans, called
through the C ABI: two calls in a row, the second with fewer samples than the
first, and the size limit of the array."""
import ctypes

import numpy as np
import pytest

from nudft import rel_l2
from paper_1710_03197_amd import _lib, data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAX_M = 1 << 21  # samples the static array holds per buffer


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _call(name, plan, iters, w):
    lib = _lib.load()
    st = getattr(lib, name)(plan.handle, int(iters), ctypes.c_void_p(w.data_ptr()),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _weights(name, plan, iters):
    w = torch.ones(plan.M, dtype=torch.float32, device=plan.device)
    _lib.check(_call(name, plan, iters, w), name)
    torch.cuda.synchronize()
    return w.cpu().numpy()


CASES = [
    # first call: the full 2D 256^2 golden-angle workload (131072 samples)
    ("2d golden radial 256", lambda: (data.config2()["om"], (256, 256)), 6),
    # second call, fewer samples: a 3D koosh ball (64 spokes x 24 readout)
    ("3d koosh 16", lambda: (data.koosh_ball_3d(64, 24), (16, 16, 16)), 4),
]


def test_noalloc_matches_allocating_entry_point_twice(dev):
    from paper_1710_03197_amd import Plan
    sizes = []
    for name, make, iters in CASES:
        om, N = make()
        K = tuple(2 * n for n in N)
        sizes.append(om.shape[0])
        print(f"{name}: N={N} M={om.shape[0]} iters={iters}", flush=True)
        with Plan(torch.from_numpy(np.ascontiguousarray(om)).to(dev), N, K, 6) as p:
            ref = _weights("nufft_density_compensation", p, iters)
            got = _weights("nufft_density_compensation_noalloc", p, iters)
        e = rel_l2(got, ref)
        print(f"{name}: no-alloc vs allocating rel L2 {e:.2e}, max |diff| {np.abs(got - ref).max():.2e}",
              flush=True)
        assert np.all(np.isfinite(got))
        assert e <= 1e-6
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_more_samples_than_the_array_holds(dev):
    from paper_1710_03197_amd import Plan
    om = np.random.default_rng(7).uniform(-np.pi, np.pi, (MAX_M + 1, 1)).astype(np.float32)
    with Plan(torch.from_numpy(om).to(dev), (64,), (128,), 6) as p:
        w = torch.ones(p.M, dtype=torch.float32, device=dev)
        st = _call("nufft_density_compensation_noalloc", p, 2, w)
        assert st == -1  # NUFFT_ERR_INVALID_ARG
        assert b"exceeds" in _lib.load().nufft_last_error()
        torch.cuda.synchronize()
        assert torch.all(w == 1).item()  # nothing ran
