"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, validates arguments before touching a
device, rejects bad handles, and its kernel fit matches the oracle's kernel."""
import ctypes

import numpy as np
import pytest

from paper_1710_03197_amd import _lib

lib = _lib.load()


def _plan(d, N, K, J, M):
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * max(d, 1))(*N)
    k = (ctypes.c_int64 * max(d, 1))(*K)
    st = lib.nufft_plan(d, n, k, J, M, ctypes.c_void_p(), ctypes.c_void_p(), ctypes.byref(h))
    return st, h


def test_exports_every_declared_symbol():
    names = _lib.declared_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/nufft_mi355x.h but not exported"


def test_status_strings():
    for code in range(-7, 1):
        assert lib.nufft_status_string(code)
    assert lib.nufft_status_string(-1) == b"invalid argument"
    assert lib.nufft_status_string(99) == b"unknown status"


@pytest.mark.parametrize("d,N,K,J,M,code", [
    (0, (8,), (16,), 6, 10, -1),           # d out of range
    (4, (8,), (16,), 6, 10, -1),
    (2, (7, 8), (16, 16), 6, 0, -1),       # odd N
    (2, (8, 8), (6, 16), 6, 0, -1),        # K < N
    (2, (8, 8), (17, 16), 6, 0, -1),       # odd K
    (2, (8, 8), (16, 16), 1, 0, -1),       # J too small
    (2, (8, 8), (16, 16), 17, 0, -1),      # J too large
    (1, (8,), (16,), 6, -5, -1),           # negative M
    (1, (8,), (16,), 6, 10, -1),           # om NULL with M > 0
    (1, (8,), (14,), 6, 0, -7),            # prime factor 7
    (1, (8,), (8192,), 6, 0, -7),          # K above 4096
])
def test_plan_argument_validation(d, N, K, J, M, code):
    st, h = _plan(d, N, K, J, M)
    assert st == code
    assert h.value is None
    assert lib.nufft_last_error()


def test_plan_without_device_reports_no_device():
    if lib.nufft_device_count() > 0:
        pytest.skip("a device is visible")
    st, h = _plan(2, (8, 8), (16, 16), 6, 0)
    assert st == -2
    assert b"device" in lib.nufft_last_error()


def test_bad_handles():
    assert lib.nufft_destroy(ctypes.c_void_p()) == -5
    junk = ctypes.create_string_buffer(256)
    assert lib.nufft_destroy(ctypes.cast(junk, ctypes.c_void_p)) == -5
    assert lib.nufft_forward(ctypes.cast(junk, ctypes.c_void_p), None, None, None) == -5
    assert lib.nufft_adjoint(None, None, None, None) == -5
    assert lib.nufft_plan_info(None, None, None, None, None, None, None) == -5


@pytest.mark.parametrize("J,sigma", [(6, 2.0), (4, 2.0), (7, 2.0), (8, 1.5), (16, 2.0), (2, 2.0)])
def test_kernel_fit_matches_oracle_kernel(orc, J, sigma):
    """The float32 per-tap polynomials the GPU evaluates agree with the oracle's
    float64 Kaiser-Bessel kernel to ~1e-7 of its peak."""
    from paper_1710_03197_amd.plan import kernel_weights_host
    f = np.linspace(0.0, 1.0, 257, endpoint=False)
    w, dw = kernel_weights_host(J, sigma, f)
    beta = orc.kb_beta(J, sigma)
    p0 = orc.kb_phi(0.0, J, beta)
    ref = np.array([[orc.kb_phi(fi + J / 2 - 1 - j, J, beta) for j in range(J)] for fi in f])
    dref = np.array([[orc.kb_dphi(fi + J / 2 - 1 - j, J, beta) for j in range(J)] for fi in f])
    assert np.abs(w - ref).max() < 4e-7 * p0
    assert np.abs(dw - dref).max() < 4e-7 * np.abs(dref).max()


def test_kernel_fit_rejects_bad_arguments():
    f = np.zeros(3)
    w = np.zeros(3 * 6)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.nufft_kernel_weights_host(1, 2.0, 3, f.ctypes.data_as(dp), w.ctypes.data_as(dp), None) == -1
    assert lib.nufft_kernel_weights_host(6, 0.5, 3, f.ctypes.data_as(dp), w.ctypes.data_as(dp), None) == -1


def test_new_entry_points_reject_bad_handles():
    """The Toeplitz operator, density compensation and the TV kernels validate
    their handles and arguments on the host (no device is touched)."""
    vp = ctypes.c_void_p
    assert lib.nufft_toeplitz_apply(vp(), 1, vp(), vp(), vp()) == -5
    assert lib.nufft_toeplitz_destroy(vp()) == -5
    assert lib.nufft_toeplitz_destroy(vp(0x1234)) == -5
    out = vp()
    assert lib.nufft_toeplitz_plan(vp(), vp(), vp(), ctypes.byref(out)) == -5
    assert lib.nufft_toeplitz_plan(vp(0x10), vp(), vp(), ctypes.byref(out)) == -5
    assert lib.nufft_density_compensation(vp(), 3, vp(), vp()) == -5
    assert lib.nufft_density_compensation_noalloc(vp(), 3, vp(), vp()) == -5
    assert lib.nufft_density_compensation_noalloc(vp(0x1234), 3, vp(), vp()) == -5
    assert lib.nufft_grad_points_batched(vp(), 2, vp(), vp(), vp(), vp()) == -5
    assert lib.nufft_set_points(vp(), vp(), vp()) == -5


@pytest.mark.parametrize("d,N,t,code", [
    (0, (8,), 1.0, -1),
    (4, (8, 8, 8, 8), 1.0, -1),
    (2, (8, 0), 1.0, -1),
    (2, (8, 8), -1.0, -1),
    (2, (8, 8), float("nan"), -1),
])
def test_tv_kernels_validate_arguments(d, N, t, code):
    n = (ctypes.c_int64 * len(N))(*N)
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    f = ctypes.c_float
    assert lib.nufft_tv_shrink(d, n, dummy, dummy, dummy, f(t), ctypes.c_void_p()) == code
    if t >= 0:  # the threshold only matters to the shrink calls
        assert lib.nufft_tv_normal(d, n, f(1.0), dummy, f(1.0), dummy, dummy, ctypes.c_void_p()) == code
        assert lib.nufft_tv_rhs(d, n, f(1.0), dummy, None, None, f(1.0), dummy, dummy, dummy,
                                ctypes.c_void_p()) == code


def test_tv_kernels_reject_null_and_half_lad_arguments():
    n = (ctypes.c_int64 * 2)(8, 8)
    dummy = ctypes.c_void_p(0x1000)
    f = ctypes.c_float
    assert lib.nufft_tv_shrink(2, n, None, dummy, dummy, f(1.0), None) == -1
    assert lib.nufft_tv_normal(2, n, f(1.0), None, f(1.0), dummy, dummy, None) == -1
    # df without bf (or the reverse) is an error
    assert lib.nufft_tv_rhs(2, n, f(1.0), dummy, dummy, None, f(1.0), dummy, dummy, dummy, None) == -1
    assert lib.nufft_bregman_shrink(ctypes.c_int64(-1), dummy, dummy, dummy, f(1.0), None) == -1
    assert lib.nufft_bregman_shrink(ctypes.c_int64(0), None, None, None, f(1.0), None) == 0
    assert lib.nufft_bregman_shrink(ctypes.c_int64(4), dummy, dummy, dummy, f(-2.0), None) == -1


def test_options_struct_matches_header():
    """The Python binding's nufft_options_t has the header's fields, in order,
    with the same element counts (all int), and the same size."""
    import re
    text = open(_lib.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} nufft_options_t;", text).group(1)
    fields = []
    for decl in filter(None, (x.strip() for x in body.split(";"))):
        m = re.fullmatch(r"int\s+(\w+)(?:\[(\d+)\])?", decl)
        assert m, decl
        fields.append((m.group(1), int(m.group(2) or 1)))
    py = [(name, getattr(ct, "_length_", 1)) for name, ct in _lib.PlanOptions._fields_]
    assert py == fields
    assert ctypes.sizeof(_lib.PlanOptions) == 4 * sum(n for _, n in fields)
