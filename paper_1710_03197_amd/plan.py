"""Python face of the C ABI: a NUFFT plan over torch device tensors.

Every method marshals tensor pointers and the current HIP stream into the
library; all arithmetic runs in the library's HIP kernels.  Images are
complex64 [*N] (C order), samples complex64 [M], trajectories float32 [M, d]
in radians (paper Section 2.1: A = V F S and A^H = S^H F^H V^H).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, dtype, shape, name: str, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def options_struct(options: dict | None) -> "_lib.PlanOptions":
    """nufft_options_t from a dict of plan options (missing keys: 0 = default)."""
    options = options or {}
    opt = _lib.PlanOptions()
    for a, t in enumerate(options.get("tile", ())[:3]):
        opt.tile[a] = int(t)
    opt.grid_chunk = int(options.get("grid_chunk", 0))
    opt.fft_groups = int(options.get("fft_groups", 0))
    opt.interp_direct = int(bool(options.get("interp_direct", 0)))
    opt.presort = int(options.get("presort", 0))
    opt.fuse_reduce = int(options.get("fuse_reduce", 0))
    opt.grid_mfma = int(options.get("grid_mfma", 0))
    opt.interp_merge = int(options.get("interp_merge", 0))
    opt.weight_table = int(options.get("weight_table", 0))
    opt.fft_radix = int(options.get("fft_radix", 0))
    opt.grid_waves = int(options.get("grid_waves", 0))
    interp = options.get("interpolator", 0)
    opt.interpolator = {"kb": 0, "kaiser-bessel": 0, "minmax": 1, "min-max": 1}.get(interp, interp) \
        if isinstance(interp, str) else int(interp)
    return opt


class Plan:
    """NUFFT plan for image size N, oversampled grid K, J taps per axis and the
    trajectory `om` (float32 [M, d] on a HIP device).  Optional `coils`
    (complex64 [C, *N]) switch on coil mode (paper Section 2.2)."""

    def __init__(self, om: torch.Tensor, N, K=None, J: int = 6, coils: torch.Tensor | None = None,
                 options: dict | None = None):
        N = tuple(int(n) for n in N)
        d = len(N)
        K = tuple(2 * n for n in N) if K is None else tuple(int(k) for k in K)
        if om.dim() != 2 or om.shape[1] != d:
            raise ValueError(f"om must be [M, {d}]")
        self.device = om.device
        if self.device.type != "cuda":
            raise ValueError("om must live on a HIP device")
        om = om.contiguous()
        self.N, self.K, self.J, self.d = N, K, int(J), d
        self.M = int(om.shape[0])
        self.C = 0
        self.generation = 0  # trajectories re-binned into this plan (set_points)
        self._handle = ctypes.c_void_p()
        n_arr = (ctypes.c_int64 * d)(*N)
        k_arr = (ctypes.c_int64 * d)(*K)
        self.options = dict(options or {})
        opt = options_struct(self.options)
        with torch.cuda.device(self.device):
            _lib.call("nufft_plan_ex", d, n_arr, k_arr, self.J, self.M,
                      _ptr(om) if self.M else ctypes.c_void_p(), ctypes.byref(opt), _stream(self.device),
                      ctypes.byref(self._handle))
        if coils is not None:
            self.set_coils(coils)

    # ------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            _lib.call("nufft_destroy", self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        if not self._handle.value:
            raise RuntimeError("plan is closed")
        return self._handle

    # ------------------------------------------------------------ configuration
    def set_points(self, om: torch.Tensor):
        """Re-bin the plan for a new trajectory (same M).  Graphs captured from
        this plan before the call must not be replayed after it."""
        _need(om, torch.float32, (self.M, self.d), "om", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_set_points", self.handle, _ptr(om), _stream(self.device))
        self.generation += 1

    def set_coils(self, coils: torch.Tensor | None):
        with torch.cuda.device(self.device):
            torch.cuda.current_stream(self.device).synchronize()
            if coils is None:
                _lib.call("nufft_set_coils", self.handle, 0, ctypes.c_void_p())
                self.C = 0
                return
            C = int(coils.shape[0])
            _need(coils, torch.complex64, (C,) + self.N, "coils", self.device)
            _lib.call("nufft_set_coils", self.handle, C, _ptr(coils))
            self.C = C

    def reserve(self, B: int):
        with torch.cuda.device(self.device):
            _lib.call("nufft_reserve", self.handle, int(B))

    def info(self) -> dict:
        beta = (ctypes.c_double * 3)()
        deg = ctypes.c_int()
        tile = (ctypes.c_int * 3)()
        nb, ni, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.call("nufft_plan_info", self.handle, beta, ctypes.byref(deg), tile, ctypes.byref(nb),
                  ctypes.byref(ni), ctypes.byref(ws))
        return dict(beta=list(beta)[:self.d], poly_degree=deg.value, tile=list(tile)[:self.d],
                    n_bins=nb.value, n_items=ni.value, workspace_bytes=ws.value)

    def timing(self, enable: bool):
        """Start (True) or stop (False) per-kernel event timing; both discard
        what was collected."""
        _lib.call("nufft_timing_enable", self.handle, 1 if enable else 0)

    def timing_report(self) -> dict:
        """{kernel name: (launches, total ms)} for kernels launched since
        timing(True); waits for the recorded events."""
        out = {}
        lib = _lib.load()
        for k in range(lib.nufft_timing_kernels()):
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            _lib.call("nufft_timing_read", self.handle, k, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms))
            if n.value:
                out[name.value.decode()] = (n.value, ms.value)
        return out

    # ------------------------------------------------------------ shapes
    def _yshape(self, B=None):
        s = (self.M,)
        if self.C:
            s = (self.C,) + s
        if B is not None:
            s = (B,) + s
        return s

    # ------------------------------------------------------------ transforms
    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """y = A x (in coil mode y[i] = A (c_i x), shape [C, M])."""
        _need(x, torch.complex64, self.N, "x", self.device)
        y = out if out is not None else torch.empty(self._yshape(), dtype=torch.complex64, device=self.device)
        _need(y, torch.complex64, self._yshape(), "y", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_forward", self.handle, _ptr(x), _ptr(y), _stream(self.device))
        return y

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """x = A^H y (in coil mode sum_i conj(c_i) A^H y[i])."""
        _need(y, torch.complex64, self._yshape(), "y", self.device)
        x = out if out is not None else torch.empty(self.N, dtype=torch.complex64, device=self.device)
        _need(x, torch.complex64, self.N, "x", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_adjoint", self.handle, _ptr(y), _ptr(x), _stream(self.device))
        return x

    def forward_batched(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        B = int(x.shape[0])
        _need(x, torch.complex64, (B,) + self.N, "x", self.device)
        y = out if out is not None else torch.empty(self._yshape(B), dtype=torch.complex64, device=self.device)
        _need(y, torch.complex64, self._yshape(B), "y", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_forward_batched", self.handle, B, _ptr(x), _ptr(y), _stream(self.device))
        return y

    def adjoint_batched(self, y: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        B = int(y.shape[0])
        _need(y, torch.complex64, self._yshape(B), "y", self.device)
        x = out if out is not None else torch.empty((B,) + self.N, dtype=torch.complex64, device=self.device)
        _need(x, torch.complex64, (B,) + self.N, "x", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_adjoint_batched", self.handle, B, _ptr(y), _ptr(x), _stream(self.device))
        return x

    def grad_points(self, x: torch.Tensor, gy: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Trajectory gradient (float32 [M, d]) of a real loss through y = A(om) x,
        given gy = dL/dRe y + i dL/dIm y."""
        _need(x, torch.complex64, self.N, "x", self.device)
        _need(gy, torch.complex64, self._yshape(), "gy", self.device)
        g = out if out is not None else torch.empty((self.M, self.d), dtype=torch.float32, device=self.device)
        _need(g, torch.float32, (self.M, self.d), "gom", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_grad_points", self.handle, _ptr(x), _ptr(gy), _ptr(g), _stream(self.device))
        return g

    def grad_points_batched(self, x: torch.Tensor, gy: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Trajectory gradient summed over a batch: x [B, *N], gy [B, M] ([B, C, M]
        with coils) -> float32 [M, d]."""
        B = int(x.shape[0])
        _need(x, torch.complex64, (B,) + self.N, "x", self.device)
        _need(gy, torch.complex64, self._yshape(B), "gy", self.device)
        g = out if out is not None else torch.empty((self.M, self.d), dtype=torch.float32, device=self.device)
        _need(g, torch.float32, (self.M, self.d), "gom", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_grad_points_batched", self.handle, B, _ptr(x), _ptr(gy), _ptr(g), _stream(self.device))
        return g

    def density_compensation(self, iters: int = 10, w0: torch.Tensor | None = None,
                             form: str = "vvh") -> torch.Tensor:
        """Sampling-density weights w (float32 [M]) by `iters` Pipe-Menon steps
        from w0 (all ones by default), paper Section 2.2, Eq. pipe_density.
        form="vvh": w <- w / (V V^H w) in the library (nufft_density_compensation;
        coils ignored).  form="aah": the equation as printed, w <- w / |A A^H w|,
        composed from this plan's forward and adjoint (no coils); it does not
        settle on evenly spaced radial sampling, which is why "vvh" is the
        default."""
        w = (torch.ones(self.M, dtype=torch.float32, device=self.device) if w0 is None
             else w0.detach().to(torch.float32).clone())
        _need(w, torch.float32, (self.M,), "w", self.device)
        if form == "aah":
            if self.C:
                raise ValueError("the printed form A A^H runs on a plan without coils")
            if iters < 0:
                raise ValueError("iters must be >= 0")
            with torch.cuda.device(self.device):
                for _ in range(int(iters)):
                    u = self.forward(self.adjoint(w.to(torch.complex64))).abs()
                    w = torch.where(u != 0, w / torch.where(u != 0, u, torch.ones_like(u)), w)
            return w
        if form != "vvh":
            raise ValueError("form is 'vvh' or 'aah'")
        with torch.cuda.device(self.device):
            _lib.call("nufft_density_compensation", self.handle, int(iters), _ptr(w), _stream(self.device))
        return w

    def toeplitz(self, weights: torch.Tensor | None = None) -> "Toeplitz":
        """The normal operator A^H W A of this plan as a Toeplitz embedding."""
        return Toeplitz(self, weights)

    # ------------------------------------------------------------ stages
    def stage_fs(self, x: torch.Tensor) -> torch.Tensor:
        _need(x, torch.complex64, self.N, "x", self.device)
        G = torch.empty(self.K, dtype=torch.complex64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_stage_fs", self.handle, _ptr(x), _ptr(G), _stream(self.device))
        return G

    def stage_v(self, G: torch.Tensor) -> torch.Tensor:
        _need(G, torch.complex64, self.K, "G", self.device)
        y = torch.empty(self.M, dtype=torch.complex64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_stage_v", self.handle, _ptr(G), _ptr(y), _stream(self.device))
        return y

    def stage_vh(self, y: torch.Tensor) -> torch.Tensor:
        _need(y, torch.complex64, (self.M,), "y", self.device)
        h = torch.empty(self.K, dtype=torch.complex64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_stage_vh", self.handle, _ptr(y), _ptr(h), _stream(self.device))
        return h

    def stage_shfh(self, h: torch.Tensor) -> torch.Tensor:
        _need(h, torch.complex64, self.K, "h", self.device)
        x = torch.empty(self.N, dtype=torch.complex64, device=self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_stage_shfh", self.handle, _ptr(h), _ptr(x), _stream(self.device))
        return x


class Toeplitz:
    """The normal operator A^H W A of a plan applied through its Toeplitz
    embedding (include/nufft_mi355x.h, nufft_toeplitz_*): two FFTs of size 2N
    and a product per application, no interpolation.  `weights`: float32 [M]
    sample weights (density compensation) on the plan's device, None for 1.
    In coil mode the plan's coils at call time are applied and combined.
    Keep it closed before its plan."""

    def __init__(self, plan: Plan, weights: torch.Tensor | None = None):
        self.plan = plan
        self.N = plan.N
        self.device = plan.device
        self._handle = ctypes.c_void_p()
        if weights is not None:
            _need(weights, torch.float32, (plan.M,), "weights", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_toeplitz_plan", plan.handle, _ptr(weights) if weights is not None else None,
                      _stream(self.device), ctypes.byref(self._handle))

    def close(self):
        if self._handle:
            _lib.call("nufft_toeplitz_destroy", self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def apply(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """A^H W A x for x [N...] or a batch [B, N...]."""
        batched = x.dim() == len(self.N) + 1
        B = int(x.shape[0]) if batched else 1
        shape = ((B,) if batched else ()) + self.N
        _need(x, torch.complex64, shape, "x", self.device)
        o = out if out is not None else torch.empty(shape, dtype=torch.complex64, device=self.device)
        _need(o, torch.complex64, shape, "out", self.device)
        with torch.cuda.device(self.device):
            _lib.call("nufft_toeplitz_apply", self._handle, B, _ptr(x), _ptr(o), _stream(self.device))
        return o

    __call__ = apply


class MultiPlan:
    """P uneven problems (own N, K, M, trajectory, coils, plan options; shared d
    and J) run together: every stage is one kernel launch over the work blocks
    of all problems (nufft_multi_forward/adjoint), and the launches of one
    direction are captured into a HIP graph per set of buffers.

    problems: list of dicts with keys om (float32 [M, d] device tensor), N,
    K (default 2N), coils (complex64 [C, *N] device tensor or None) and
    options (plan options dict, or None).  tune="cache" fills a problem's
    missing options from the shipped tuning cache (autotune.SHIPPED_CACHE)
    when it holds an entry for that problem's sizes; tune="off" keeps the
    built-in defaults."""

    def __init__(self, problems, J: int = 6, tune: str = "off"):
        self.device = problems[0]["om"].device
        self.J = int(J)
        self.problems = []
        descs = (_lib.ProblemDesc * len(problems))()
        keep = []
        for i, pr in enumerate(problems):
            om = pr["om"].contiguous()
            N = tuple(int(n) for n in pr["N"])
            K = tuple(2 * n for n in N) if pr.get("K") is None else tuple(int(k) for k in pr["K"])
            d = len(N)
            coils = pr.get("coils")
            C = 0
            if coils is not None:
                coils = coils.contiguous()
                C = int(coils.shape[0])
                _need(coils, torch.complex64, (C,) + N, "coils", self.device)
            _need(om, torch.float32, (om.shape[0], d), "om", self.device)
            options = pr.get("options")
            if options is None and tune == "cache":
                from . import autotune
                options = autotune.cached_options(N, K, self.J, int(om.shape[0]), autotune.SHIPPED_CACHE, self.device,
                                                  C)
            opt = options_struct(options) if options else None
            keep += [om, coils, opt]
            desc = descs[i]
            desc.d, desc.J, desc.M, desc.C = d, self.J, int(om.shape[0]), C
            for a in range(d):
                desc.N[a] = N[a]
                desc.K[a] = K[a]
            desc.om = om.data_ptr() if om.shape[0] else None
            desc.coils = coils.data_ptr() if coils is not None else None
            desc.opt = ctypes.addressof(opt) if opt is not None else None
            self.problems.append(dict(N=N, K=K, M=int(om.shape[0]), C=C, d=d, options=dict(options or {})))
        self._handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.call("nufft_multi_plan", len(problems), descs, _stream(self.device), ctypes.byref(self._handle))
        del keep

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            _lib.call("nufft_multi_destroy", self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def launches(self) -> tuple:
        """(forward, adjoint) kernel launches per call for the last buffers
        used in each direction (-1: not called yet)."""
        f, a = ctypes.c_int64(), ctypes.c_int64()
        _lib.call("nufft_multi_info", self._handle, ctypes.byref(f), ctypes.byref(a))
        return f.value, a.value

    def yshape(self, p):
        pr = self.problems[p]
        return ((pr["C"],) if pr["C"] else ()) + (pr["M"],)

    def _ptrs(self, ts, shapes, name):
        arr = (ctypes.c_void_p * len(ts))()
        for i, (t, shp) in enumerate(zip(ts, shapes)):
            _need(t, torch.complex64, shp, f"{name}[{i}]", self.device)
            arr[i] = t.data_ptr()
        return arr

    def forward(self, xs, ys=None):
        """ys[p] = A_p xs[p] for every problem (coil mode: [C_p, M_p])."""
        P = len(self.problems)
        if ys is None:
            ys = [torch.empty(self.yshape(p), dtype=torch.complex64, device=self.device) for p in range(P)]
        xa = self._ptrs(xs, [pr["N"] for pr in self.problems], "x")
        ya = self._ptrs(ys, [self.yshape(p) for p in range(P)], "y")
        with torch.cuda.device(self.device):
            _lib.call("nufft_multi_forward", self._handle, xa, ya, _stream(self.device))
        return ys

    def adjoint(self, ys, xs=None):
        P = len(self.problems)
        if xs is None:
            xs = [torch.empty(pr["N"], dtype=torch.complex64, device=self.device) for pr in self.problems]
        ya = self._ptrs(ys, [self.yshape(p) for p in range(P)], "y")
        xa = self._ptrs(xs, [pr["N"] for pr in self.problems], "x")
        with torch.cuda.device(self.device):
            _lib.call("nufft_multi_adjoint", self._handle, ya, xa, _stream(self.device))
        return xs


def kernel_weights_host(J: int, sigma: float, f) -> tuple:
    """The per-tap weights (and derivatives) the GPU evaluates, computed on the
    host from the same polynomial fit: arrays [len(f), J]."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).ravel())
    w = np.empty((f.size, J), np.float64)
    dw = np.empty((f.size, J), np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.call("nufft_kernel_weights_host", int(J), float(sigma), f.size, f.ctypes.data_as(dp),
              w.ctypes.data_as(dp), dw.ctypes.data_as(dp))
    return w, dw


def device_count() -> int:
    return int(_lib.load().nufft_device_count())
