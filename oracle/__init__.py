"""FP64 CPU oracle for the NUFFT pair (paper Section 2.1, A = V F S and
A^H = S^H F^H V^H), with coil handling (Section 2.2, multi-coil), the
trajectory gradient and a plain conjugate-gradient driver.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the GPU
library.  Inputs are the same float32 coordinates and complex64 images the GPU
sees, widened exactly to float64 / complex128.

Pins (all in tests/test_oracle_*.py, run on the CPU):
  kb_ft ........ quadrature of kb_phi; kb_dphi ... central differences;
  fftn ......... numpy.fft.fftn, Parseval;
  forward ...... brute-force NUDFT, delta / constant image closed forms,
                 Cartesian samples reduce to numpy.fft;
  adjoint ...... <A x, y> = <x, A^H y> to 1e-12, single-sample closed form;
  grad_points .. central finite differences of the oracle loss;
  cg ........... CG on the explicit dense matrix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_nufft.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_kb_beta.restype = ctypes.c_double
    lib.orc_kb_beta.argtypes = [ctypes.c_int, ctypes.c_double]
    for f in ("orc_i0", "orc_i1_over_z"):
        getattr(lib, f).restype = ctypes.c_double
        getattr(lib, f).argtypes = [ctypes.c_double]
    for f in ("orc_kb_phi", "orc_kb_dphi", "orc_kb_ft"):
        getattr(lib, f).restype = ctypes.c_double
        getattr(lib, f).argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_toeplitz_conv.argtypes = [ctypes.c_int, _i64p, _dp, _dp, _dp]
    lib.orc_scaling.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, _dp]
    lib.orc_fftn.argtypes = [ctypes.c_int, _i64p, _dp, ctypes.c_int]
    lib.orc_fft_axis.argtypes = [ctypes.c_int, _i64p, ctypes.c_int, _dp, ctypes.c_int]
    lib.orc_pad_scale.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, _dp, _dp]
    lib.orc_crop_scale.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, _dp, _dp]
    lib.orc_interp.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp]
    lib.orc_grid.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64, _dp, _dp, _dp]
    lib.orc_forward.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64,
                                _dp, _dp, _dp, _dp, _dp]
    lib.orc_adjoint.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64,
                                _dp, _dp, _dp, _dp, _dp]
    lib.orc_grad_points.argtypes = [ctypes.c_int, _i64p, _i64p, ctypes.c_int, ctypes.c_int64,
                                    _dp, _dp, _dp, _dp]
    _lib = lib
    return lib


def _shape(v):
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int64))
    return a, a.ctypes.data_as(_i64p)


def _c128(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a, a.ctypes.data_as(_dp)


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(_dp)


def _null():
    return ctypes.cast(None, _dp)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ------------------------------------------------------------------ kernel
def kb_beta(J: int, sigma: float) -> float:
    return float(_load().orc_kb_beta(int(J), float(sigma)))


def i0(z: float) -> float:
    return float(_load().orc_i0(float(z)))


def i1_over_z(z: float) -> float:
    return float(_load().orc_i1_over_z(float(z)))


def kb_phi(t: float, J: int, beta: float) -> float:
    return float(_load().orc_kb_phi(float(t), int(J), float(beta)))


def kb_dphi(t: float, J: int, beta: float) -> float:
    return float(_load().orc_kb_dphi(float(t), int(J), float(beta)))


def kb_ft(xi: float, J: int, beta: float) -> float:
    return float(_load().orc_kb_ft(float(xi), int(J), float(beta)))


def scaling(N, K, J) -> list:
    """Per-axis scaling tables s_a(i) = 1/Phi_a((i - N_a/2)/K_a)."""
    N = list(N)
    out = np.empty(sum(N), dtype=np.float64)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_scaling(len(N), np_, kp, int(J), out.ctypes.data_as(_dp))
    res, off = [], 0
    for n_a in N:
        res.append(out[off:off + n_a].copy())
        off += n_a
    return res


# ------------------------------------------------------------------ FFT
def fftn(a, sign: int = -1) -> np.ndarray:
    """Unnormalised multi-dimensional DFT with kernel e^{sign 2 pi i q k / L}."""
    arr, p = _c128(np.array(a, dtype=np.complex128, copy=True))
    s, sp = _shape(arr.shape)
    _load().orc_fftn(arr.ndim, sp, p, int(sign))
    return arr


def fft_axis(a, axis: int, sign: int = -1) -> np.ndarray:
    arr, p = _c128(np.array(a, dtype=np.complex128, copy=True))
    s, sp = _shape(arr.shape)
    _load().orc_fft_axis(arr.ndim, sp, int(axis), p, int(sign))
    return arr


# ------------------------------------------------------------------ stages
def pad_scale(x, N, K, J) -> np.ndarray:
    d = len(N)
    xx, xp = _c128(x)
    g = np.empty(tuple(K), dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_pad_scale(d, np_, kp, int(J), xp, g.ctypes.data_as(_dp))
    return g


def crop_scale(H, N, K, J) -> np.ndarray:
    d = len(N)
    hh, hp = _c128(H)
    x = np.empty(tuple(N), dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_crop_scale(d, np_, kp, int(J), hp, x.ctypes.data_as(_dp))
    return x


def interp(G, om, N, K, J) -> np.ndarray:
    d = len(N)
    om_, omp = _f64(om)
    M = om_.shape[0]
    gg, gp = _c128(G)
    y = np.empty(M, dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_interp(d, np_, kp, int(J), M, omp, gp, y.ctypes.data_as(_dp))
    return y


def grid(y, om, N, K, J) -> np.ndarray:
    d = len(N)
    om_, omp = _f64(om)
    M = om_.shape[0]
    yy, yp = _c128(y)
    h = np.empty(tuple(K), dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_grid(d, np_, kp, int(J), M, omp, yp, h.ctypes.data_as(_dp))
    return h


# ------------------------------------------------------------------ transforms
def forward(x, om, N, K, J, stages: bool = False):
    """y = V F S x.  With stages=True also returns (g, G): the padded scaled
    image and its oversampled FFT."""
    d = len(N)
    om_, omp = _f64(om)
    M = om_.shape[0]
    xx, xp = _c128(np.asarray(x).reshape(tuple(N)))
    y = np.empty(M, dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    if stages:
        g = np.empty(tuple(K), dtype=np.complex128)
        G = np.empty(tuple(K), dtype=np.complex128)
        _load().orc_forward(d, np_, kp, int(J), M, omp, xp, y.ctypes.data_as(_dp),
                            g.ctypes.data_as(_dp), G.ctypes.data_as(_dp))
        return y, g, G
    _load().orc_forward(d, np_, kp, int(J), M, omp, xp, y.ctypes.data_as(_dp), _null(), _null())
    return y


def adjoint(y, om, N, K, J, stages: bool = False):
    """x = S^H F^H V^H y.  With stages=True also returns (h, H): the gridded
    samples and their inverse oversampled FFT."""
    d = len(N)
    om_, omp = _f64(om)
    M = om_.shape[0]
    yy, yp = _c128(y)
    x = np.empty(tuple(N), dtype=np.complex128)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    if stages:
        h = np.empty(tuple(K), dtype=np.complex128)
        H = np.empty(tuple(K), dtype=np.complex128)
        _load().orc_adjoint(d, np_, kp, int(J), M, omp, yp, x.ctypes.data_as(_dp),
                            h.ctypes.data_as(_dp), H.ctypes.data_as(_dp))
        return x, h, H
    _load().orc_adjoint(d, np_, kp, int(J), M, omp, yp, x.ctypes.data_as(_dp), _null(), _null())
    return x


def forward_grid(x, N, K, J) -> np.ndarray:
    """G = F S x (the oversampled spectrum the interpolator reads)."""
    return fftn(pad_scale(x, N, K, J), -1)


def grad_points(G, gy, om, N, K, J, out=None) -> np.ndarray:
    """Trajectory gradient of a real loss through y = V(omega) G, given the
    torch-convention gradient gy of y.  Adds into `out` when given."""
    d = len(N)
    om_, omp = _f64(om)
    M = om_.shape[0]
    gg, gp = _c128(G)
    yy, yp = _c128(gy)
    if out is None:
        out = np.zeros((M, d), dtype=np.float64)
    o = np.ascontiguousarray(out, dtype=np.float64)
    n, np_ = _shape(N)
    k, kp = _shape(K)
    _load().orc_grad_points(d, np_, kp, int(J), M, omp, gp, yp, o.ctypes.data_as(_dp))
    return o


# ------------------------------------------------------------------ coils (Section 2.2)
def forward_coils(x, coils, om, N, K, J) -> np.ndarray:
    """y_i = A (c_i * x) for every coil i."""
    return np.stack([forward(np.asarray(c, np.complex128) * np.asarray(x, np.complex128),
                             om, N, K, J) for c in coils])


def adjoint_coils(ys, coils, om, N, K, J) -> np.ndarray:
    """sum_i conj(c_i) * A^H y_i."""
    acc = np.zeros(tuple(N), dtype=np.complex128)
    for c, y in zip(coils, ys):
        acc += np.conj(np.asarray(c, np.complex128)) * adjoint(y, om, N, K, J)
    return acc


def loss_and_grads(x, om, coils, target_y, N, K, J):
    """L = sum_i ||A(c_i x) - y_i||^2 with its torch-convention image gradient
    2 sum_i conj(c_i) A^H r_i and the trajectory gradient (float64 [M, d])."""
    x = np.asarray(x, np.complex128)
    M = np.asarray(om).shape[0]
    L = 0.0
    gx = np.zeros(tuple(N), np.complex128)
    gom = np.zeros((M, len(N)), np.float64)
    for c, yt in zip(coils, target_y):
        cx = np.asarray(c, np.complex128) * x
        G = forward_grid(cx, N, K, J)
        y = interp(G, om, N, K, J)
        r = y - np.asarray(yt, np.complex128)
        L += float(np.vdot(r, r).real)
        gy = 2.0 * r
        gx += np.conj(np.asarray(c, np.complex128)) * adjoint(gy, om, N, K, J)
        grad_points(G, gy, om, N, K, J, out=gom)
    return L, gx, gom


# ------------------------------------------------------------------ Toeplitz normal operator
def toeplitz_psf(om, N, K, J, w=None) -> np.ndarray:
    """Point-spread function of A^H W A (paper Section 2.1, "Self-adjoint
    NUFFT"): p[Delta] = sum_m w_m e^{+i omega_m . Delta} for Delta in
    [-N, N)^d, stored centred (index Delta + N, shape 2N).  Computed the way
    the method does: the adjoint NUFFT with image size 2N and grid 2K (same
    oversampling and J) applied to the weights (w = 1 when None)."""
    N2 = tuple(2 * int(n) for n in N)
    K2 = tuple(2 * int(k) for k in K)
    M = np.asarray(om).shape[0]
    wv = np.ones(M) if w is None else np.asarray(w, np.float64)
    return adjoint(wv.astype(np.complex128), om, N2, K2, J)


def toeplitz_conv(p, x, N) -> np.ndarray:
    """out[n] = sum_{n'} p[n - n'] x[n'] over the image (direct sum)."""
    d = len(N)
    pp, ppp = _c128(np.asarray(p).reshape(tuple(2 * int(n) for n in N)))
    xx, xp = _c128(np.asarray(x).reshape(tuple(N)))
    out = np.empty(tuple(N), dtype=np.complex128)
    n, np_ = _shape(N)
    _load().orc_toeplitz_conv(d, np_, ppp, xp, out.ctypes.data_as(_dp))
    return out


def toeplitz_conv_fft(p, x, N) -> np.ndarray:
    """The same product through the circulant embedding: place p at
    Delta mod 2N and x at n mod 2N, multiply the (oracle) FFTs, invert,
    crop, divide by prod(2N).  Used where the direct sum is too slow; pinned
    against it on small sizes."""
    N = tuple(int(n) for n in N)
    P = tuple(2 * n for n in N)
    pc = np.asarray(p, np.complex128).reshape(P)
    pm = pc
    for a, n in enumerate(N):
        pm = np.roll(pm, -n, axis=a)          # centred index Delta + N -> Delta mod 2N
    xe = np.zeros(P, np.complex128)
    xe[tuple(slice(0, n) for n in N)] = np.asarray(x, np.complex128).reshape(N)
    for a, n in enumerate(N):
        xe = np.roll(xe, -(n // 2), axis=a)   # image index i -> (i - N/2) mod 2N
    z = fftn(fftn(pm, -1) * fftn(xe, -1), +1) / float(np.prod(P))
    for a, n in enumerate(N):
        z = np.roll(z, n // 2, axis=a)
    return z[tuple(slice(0, n) for n in N)]


def toeplitz_normal(x, om, N, K, J, w=None, fft: bool = False) -> np.ndarray:
    """A^H W A x by the Toeplitz embedding (PSF from the oracle adjoint)."""
    p = toeplitz_psf(om, N, K, J, w)
    return (toeplitz_conv_fft if fft else toeplitz_conv)(p, x, N)


# ------------------------------------------------------------------ density compensation
# Paper Section 2.2, "Density compensation and gridding", Eq. pipe_density:
# w_{i+1} = w_i / (A A^H w_i), after Pipe and Menon.  Two functions:
#   density_compensation_aah  the equation as printed, with the whole pair A;
#   density_compensation_vvh  the reading the GPU library builds: A A^H
#                             replaced by the interpolator product V V^H.
# Why the reading: on an evenly spaced radial trajectory the printed map
# does not settle in float64 -- its fixed-point residual |A A^H w - 1| grows
# over the iterations and the spread of the weights grows by orders of
# magnitude (tests/test_oracle_density.py measures both) -- while the V V^H
# iteration approaches its fixed point monotonically.
def density_compensation_aah(om, N, K, J, iters: int, w0=None, form: str = "modulus") -> np.ndarray:
    """The printed iteration w <- w / (A A^H w) elementwise, from w0 (ones by
    default), A the oracle forward and A^H its adjoint.  For real w the
    product A A^H w is complex (the image index range [-N/2, N/2) is not
    symmetric about 0), so the quotient has two readings: form="modulus"
    divides by |A A^H w| and keeps the weights real; form="complex" divides by
    the complex value (complex weights).  A zero entry leaves w_m unchanged."""
    if form not in ("modulus", "complex"):
        raise ValueError("form is 'modulus' or 'complex'")
    M = np.asarray(om).shape[0]
    w = np.ones(M) if w0 is None else np.asarray(w0).copy()
    if form == "complex":
        w = w.astype(np.complex128)
    for _ in range(iters):
        u = forward(adjoint(np.asarray(w, np.complex128), om, N, K, J), om, N, K, J)
        if form == "modulus":
            u = np.abs(u)
        w = np.where(u != 0, w / np.where(u != 0, u, 1.0), w)
    return w


def density_compensation_vvh(om, N, K, J, iters: int, w0=None) -> np.ndarray:
    """w <- w / (V V^H w) elementwise, from w0 (ones by default), V the oracle
    interpolator and V^H its gridding with the kernel normalised to peak 1:
    Pipe and Menon's iteration, which divides by the gridding kernel's
    convolution at the samples.  For positive w the product is real and
    positive; the modulus only removes float64 rounding in the imaginary
    part."""
    M = np.asarray(om).shape[0]
    c2 = 1.0
    for n, k in zip(N, K):
        c2 *= i0(kb_beta(J, k / n)) ** 2
    w = np.ones(M) if w0 is None else np.asarray(w0, np.float64).copy()
    for _ in range(iters):
        u = np.abs(interp(grid(w.astype(np.complex128), om, N, K, J), om, N, K, J)) / c2
        w = np.where(u > 0, w / np.where(u > 0, u, 1.0), w)
    return w


# ------------------------------------------------------------------ CG
def cg(apply_normal, b, iters: int, x0=None):
    """Conjugate gradient on the Hermitian positive semi-definite system
    N x = b, x0 = 0 unless given, <a, b> = sum conj(a) b, a fixed number of
    iterations, no preconditioner, no restart.  Returns (x, residual norms
    per iteration)."""
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, np.complex128).copy()
    r = b.copy() if x0 is None else b - apply_normal(x)
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    hist = [np.sqrt(rr)]
    for _ in range(iters):
        Ap = apply_normal(p)
        pAp = float(np.vdot(p, Ap).real)
        if pAp == 0.0:
            break
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.vdot(r, r).real)
        hist.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, np.array(hist)


def cg_nufft(y, om, N, K, J, iters: int = 30):
    """CG on A^H A x = A^H y with the oracle pair."""
    b = adjoint(y, om, N, K, J)
    return cg(lambda p: adjoint(forward(p, om, N, K, J), om, N, K, J), b, iters)


# ------------------------------------------------------------------ L1TV solvers
# Paper Section 2.2, "Iterative NUFFT": image gradient by one-sided
# differences with wrap-around (Eq. of the image gradient), TV(x) = sum over
# axes of |grad_a x| (Eq. TV), and the variable-splitting (split Bregman)
# iterations of L1TV-OLS and L1TV-LAD as printed there.
def tv_grad(x, axis: int) -> np.ndarray:
    """grad_a x = x(..., i_a + 1, ...) - x(..., i_a, ...), periodic."""
    return np.roll(x, -1, axis=axis) - x


def tv_grad_t(g, axis: int) -> np.ndarray:
    """The adjoint of tv_grad: g(..., i_a - 1, ...) - g(..., i_a, ...)."""
    return np.roll(g, 1, axis=axis) - g


def shrink(z, t: float) -> np.ndarray:
    """Soft threshold of complex values: z / |z| * max(|z| - t, 0)."""
    z = np.asarray(z, np.complex128)
    a = np.abs(z)
    scale = np.where(a > t, (a - t) / np.where(a > 0, a, 1.0), 0.0)
    return z * scale


def tv_norm(x) -> float:
    """TV(x) = sum over axes and pixels of |grad_a x|."""
    return float(sum(np.abs(tv_grad(x, a)).sum() for a in range(np.ndim(x))))


def l1tv(y, om, N, K, J, mu: float, lam: float, outer: int, inner: int, cg_iters: int, lad: bool = False):
    """L1TV-OLS (lad=False) or L1TV-LAD (lad=True) reconstruction.

    K = mu A^H A + lam sum_a grad_a^T grad_a.  Inner iterations:
      rhs = mu (A^H y^k [+ d_f - b_f]) + lam sum_a grad_a^T (d_a - b_a)
      x = K^-1 rhs   (cg_iters CG iterations from the current x)
      d_a = shrink(grad_a x + b_a, 1/lam);  b_a += grad_a x - d_a
      LAD: r = A^H A x - A^H y;  d_f = shrink(r + b_f, 1/mu);  b_f += r - d_f
    Outer iteration: A^H y^{k+1} = A^H y^k + A^H y - A^H A x.
    (The printed d_f update adds b_y^k; it is read as b_f^k, the Bregman
    variable of the same term.)  Returns x."""
    N = tuple(int(n) for n in N)
    d = len(N)
    AH = lambda v: adjoint(v, om, N, K, J)
    AHA = lambda v: adjoint(forward(v, om, N, K, J), om, N, K, J)
    ahy = AH(np.asarray(y, np.complex128))
    ahyk = ahy.copy()
    x = np.zeros(N, np.complex128)
    dd = [np.zeros(N, np.complex128) for _ in range(d)]
    bb = [np.zeros(N, np.complex128) for _ in range(d)]
    df = np.zeros(N, np.complex128)
    bf = np.zeros(N, np.complex128)

    def Kop(v):
        out = mu * AHA(v)
        for a in range(d):
            out = out + lam * tv_grad_t(tv_grad(v, a), a)
        return out

    for _ in range(outer):
        for _ in range(inner):
            rhs = mu * (ahyk + (df - bf if lad else 0.0))
            for a in range(d):
                rhs = rhs + lam * tv_grad_t(dd[a] - bb[a], a)
            x, _ = cg(Kop, rhs, cg_iters, x0=x)
            for a in range(d):
                z = tv_grad(x, a) + bb[a]
                dd[a] = shrink(z, 1.0 / lam)
                bb[a] = z - dd[a]
            if lad:
                z = AHA(x) - ahy + bf
                df = shrink(z, 1.0 / mu)
                bf = z - df
        ahyk = ahyk + ahy - AHA(x)
    return x


# ------------------------------------------------------------------ min-max interpolator
# The paper's default interpolator (Section 2.1 "Interpolation", after Fessler
# and Sutton): for a sample at u = omega K / (2 pi) with first tap k0 (the
# same window as the Kaiser-Bessel path), the J coefficients c minimise the
# worst-case error over unit-norm images,
#   || e^{-i omega n} - s_n sum_j c_j e^{-i gamma (k0 + j) n} ||_2 over n,
# gamma = 2 pi / K, i.e. c = T^-1 r with
#   T_jl = sum_n s_n^2 e^{i gamma (j - l) n},   r_j = sum_n s_n e^{-i gamma t_j n},
# t_j = u - k0 - j, n over the image range [-N/2, N/2).  Scaling factors
# (reading): the Kaiser-Bessel ones taken at the half-integer centres,
# s_n = 1 / Phi((n + 1/2) / K), which makes the range of n + 1/2 symmetric.
def minmax_scaling(N: int, K: int, J: int) -> np.ndarray:
    beta = kb_beta(J, K / N)
    n = np.arange(N) - N // 2
    return np.array([1.0 / kb_ft((v + 0.5) / K, J, beta) for v in n])


def minmax_coefs(om_a, N: int, K: int, J: int):
    """Per sample of one axis: (k0, c) with c complex [M, J] = T^-1 r."""
    om_a = np.asarray(om_a, np.float64)
    s = minmax_scaling(N, K, J)
    n = np.arange(N) - N // 2
    g = 2.0 * np.pi / K
    jj = np.arange(J)
    T = (s[None, None, :] ** 2 * np.exp(1j * g * (jj[:, None, None] - jj[None, :, None]) * n[None, None, :])).sum(-1)
    u = om_a * (K / (2.0 * np.pi))
    k0 = np.floor(u - J / 2.0) + 1.0
    t = u[:, None] - k0[:, None] - jj[None, :]                      # [M, J]
    r = (s[None, None, :] * np.exp(-1j * g * t[:, :, None] * n[None, None, :])).sum(-1)   # [M, J]
    c = np.linalg.solve(T[None], r[..., None])[..., 0]
    return k0.astype(np.int64), c


def _minmax_taps(om, N, K, J):
    d = len(N)
    per = [minmax_coefs(np.asarray(om)[:, a], N[a], K[a], J) for a in range(d)]
    M = np.asarray(om).shape[0]
    idx = np.zeros((M,) + (J,) * d, np.int64)
    w = np.ones((M,) + (J,) * d, np.complex128)
    for a in range(d):
        k0, c = per[a]
        shape = [M] + [1] * d
        shape[a + 1] = J
        kk = (k0[:, None] + np.arange(J)[None, :]) % K[a]
        idx = idx * K[a] + kk.reshape(shape)
        w = w * c.reshape(shape)
    return idx.reshape(M, -1), w.reshape(M, -1)


def minmax_forward(x, om, N, K, J) -> np.ndarray:
    """y = V_mm F S_mm x: scale by the min-max scaling factors, zero-pad and
    FFT (as the Kaiser-Bessel path), interpolate with the min-max
    coefficients."""
    N = tuple(int(v) for v in N)
    S = np.ones(N)
    for a in range(len(N)):
        shape = [1] * len(N)
        shape[a] = N[a]
        S = S * minmax_scaling(N[a], K[a], J).reshape(shape)
    xs = np.asarray(x, np.complex128).reshape(N) * S
    G = np.zeros(tuple(K), np.complex128)
    G[np.ix_(*[(np.arange(n) - n // 2) % k for n, k in zip(N, K)])] = xs
    G = fftn(G, -1)
    idx, w = _minmax_taps(om, N, K, J)
    return (w * G.ravel()[idx]).sum(1)


def minmax_adjoint(y, om, N, K, J) -> np.ndarray:
    """x = S_mm^H F^H V_mm^H y (conjugate coefficients, inverse FFT, crop,
    scale)."""
    N = tuple(int(v) for v in N)
    idx, w = _minmax_taps(om, N, K, J)
    h = np.zeros(int(np.prod(K)), np.complex128)
    np.add.at(h, idx.ravel(), (np.conj(w) * np.asarray(y, np.complex128)[:, None]).ravel())
    H = fftn(h.reshape(tuple(K)), +1)
    x = H[np.ix_(*[(np.arange(n) - n // 2) % k for n, k in zip(N, K)])]
    for a in range(len(N)):
        shape = [1] * len(N)
        shape[a] = N[a]
        x = x * minmax_scaling(N[a], K[a], J).reshape(shape)
    return x
