"""ctypes loader for libnufft_mi355x.so (the C ABI in include/nufft_mi355x.h).

The library is built in-tree by paper_1710_03197_amd.build; importing this
module never falls back to anything else: a missing or unloadable library
raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnufft_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nufft_mi355x.h")

STATUS = {
    0: "NUFFT_OK",
    -1: "NUFFT_ERR_INVALID_ARG",
    -2: "NUFFT_ERR_NO_DEVICE",
    -3: "NUFFT_ERR_OOM",
    -4: "NUFFT_ERR_HIP",
    -5: "NUFFT_ERR_BAD_PLAN",
    -6: "NUFFT_ERR_NONFINITE",
    -7: "NUFFT_ERR_UNSUPPORTED",
}


class NufftError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{func} failed with {self.code}: {detail}")


_lib = None


class PlanOptions(ctypes.Structure):
    """nufft_options_t of include/nufft_mi355x.h (0 = default)."""
    _fields_ = [("tile", ctypes.c_int * 3), ("grid_chunk", ctypes.c_int), ("fft_groups", ctypes.c_int),
                ("interp_direct", ctypes.c_int), ("presort", ctypes.c_int),
                ("fuse_reduce", ctypes.c_int), ("grid_mfma", ctypes.c_int), ("interpolator", ctypes.c_int),
                ("interp_merge", ctypes.c_int), ("weight_table", ctypes.c_int), ("fft_radix", ctypes.c_int),
                ("grid_waves", ctypes.c_int), ("reserved", ctypes.c_int * 2)]


class ProblemDesc(ctypes.Structure):
    """nufft_problem_t of include/nufft_mi355x.h."""
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int64 * 3), ("K", ctypes.c_int64 * 3),
                ("J", ctypes.c_int), ("M", ctypes.c_int64), ("om", ctypes.c_void_p),
                ("C", ctypes.c_int), ("coils", ctypes.c_void_p), ("opt", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "nufft_plan": [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64, _vp, _vp, ctypes.POINTER(_vp)],
    "nufft_plan_ex": [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64, _vp, ctypes.POINTER(PlanOptions),
                      _vp, ctypes.POINTER(_vp)],
    "nufft_set_points": [_vp, _vp, _vp],
    "nufft_set_coils": [_vp, ctypes.c_int, _vp],
    "nufft_reserve": [_vp, ctypes.c_int],
    "nufft_forward": [_vp, _vp, _vp, _vp],
    "nufft_adjoint": [_vp, _vp, _vp, _vp],
    "nufft_forward_batched": [_vp, ctypes.c_int, _vp, _vp, _vp],
    "nufft_adjoint_batched": [_vp, ctypes.c_int, _vp, _vp, _vp],
    "nufft_grad_points": [_vp, _vp, _vp, _vp, _vp],
    "nufft_grad_points_batched": [_vp, ctypes.c_int, _vp, _vp, _vp, _vp],
    "nufft_stage_fs": [_vp, _vp, _vp, _vp],
    "nufft_stage_v": [_vp, _vp, _vp, _vp],
    "nufft_stage_vh": [_vp, _vp, _vp, _vp],
    "nufft_stage_shfh": [_vp, _vp, _vp, _vp],
    "nufft_plan_info": [_vp, _dp, _ip, _ip, _i64p, _i64p, _i64p],
    "nufft_kernel_weights_host": [ctypes.c_int, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp],
    "nufft_destroy": [_vp],
    "nufft_device_count": [],
    "nufft_timing_enable": [_vp, ctypes.c_int],
    "nufft_multi_plan": [ctypes.c_int, ctypes.POINTER(ProblemDesc), _vp, ctypes.POINTER(_vp)],
    "nufft_multi_forward": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
    "nufft_multi_adjoint": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
    "nufft_multi_info": [_vp, _i64p, _i64p],
    "nufft_multi_destroy": [_vp],
    "nufft_toeplitz_plan": [_vp, _vp, _vp, ctypes.POINTER(_vp)],
    "nufft_toeplitz_apply": [_vp, ctypes.c_int, _vp, _vp, _vp],
    "nufft_toeplitz_destroy": [_vp],
    "nufft_density_compensation": [_vp, ctypes.c_int, _vp, _vp],
    "nufft_density_compensation_noalloc": [_vp, ctypes.c_int, _vp, _vp],
    "nufft_tv_shrink": [ctypes.c_int, _i64p, _vp, _vp, _vp, ctypes.c_float, _vp],
    "nufft_tv_rhs": [ctypes.c_int, _i64p, ctypes.c_float, _vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _vp],
    "nufft_tv_normal": [ctypes.c_int, _i64p, ctypes.c_float, _vp, ctypes.c_float, _vp, _vp, _vp],
    "nufft_bregman_shrink": [ctypes.c_int64, _vp, _vp, _vp, ctypes.c_float, _vp],
    "nufft_timing_kernels": [],
    "nufft_timing_read": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), _i64p, _dp],
}


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch carries its own HIP runtime (same SONAME as /opt/rocm's); loading
    # it first makes the library bind to that one, so the process holds a
    # single HIP runtime and torch's device pointers are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1710_03197_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nufft_status_string.argtypes = [ctypes.c_int]
    lib.nufft_status_string.restype = ctypes.c_char_p
    lib.nufft_last_error.argtypes = []
    lib.nufft_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, func: str):
    if status != 0:
        detail = load().nufft_last_error().decode(errors="replace")
        raise NufftError(status, func, detail)


def call(name: str, *args):
    st = getattr(load(), name)(*args)
    check(st, name)
    return st


def declared_symbols() -> list:
    """Function names declared in include/nufft_mi355x.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nufft_[a-z0-9_]+)\s*\(", text)))
