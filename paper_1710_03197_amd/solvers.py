"""Conjugate gradient on the normal equations A^H A x = A^H y (paper Section
2.1 "Self-adjoint NUFFT", Eq. normal equation; Section 2.2 "Least square
regression"), with every operator application a forward + adjoint pair of the
library.  The vector updates are torch ops on the device with device-side
scalars, so an iteration issues no host synchronisation.
"""
from __future__ import annotations

import torch

from .plan import Plan


def _dot_re(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Re <a, b> = Re sum conj(a) b as a 0-dim float32 tensor (no host sync)."""
    return (a.real * b.real + a.imag * b.imag).sum()


def cg_normal(plan: Plan, y: torch.Tensor, iters: int = 30, x0: torch.Tensor | None = None,
              history: bool = False, normal=None):
    """`iters` CG iterations on A^H A x = A^H y, x0 = 0 by default, no
    preconditioner, no restart.  A^H A is applied as a forward + adjoint pair,
    or by `normal` (e.g. the plan's Toeplitz operator, called as
    normal(p, out=...)) when given.  Returns x (and the residual norms per
    iteration when history=True; reading them synchronises once at the end)."""
    b = plan.adjoint(y)
    ybuf = torch.empty_like(y)

    def apply(v, out):
        if normal is not None:
            return normal(v, out=out)
        plan.forward(v, out=ybuf)
        return plan.adjoint(ybuf, out=out)

    x = torch.zeros_like(b) if x0 is None else x0.clone()
    r = b.clone() if x0 is None else b - apply(x, torch.empty_like(b))
    p = r.clone()
    rr = _dot_re(r, r)
    hist = [rr.sqrt()]
    ap = torch.empty_like(b)
    for _ in range(iters):
        apply(p, ap)
        pap = _dot_re(p, ap)
        alpha = rr / pap
        x.add_(p * alpha)
        r.sub_(ap * alpha)
        rr_new = _dot_re(r, r)
        beta = rr_new / rr
        p.mul_(beta).add_(r)
        rr = rr_new
        if history:
            hist.append(rr.sqrt())
    if history:
        return x, torch.stack(hist).cpu().numpy()
    return x


# ------------------------------------------------------------ L1TV (split Bregman)
# Paper Section 2.2, "Iterative NUFFT": L1TV-OLS and L1TV-LAD.  The image-
# domain steps (gradient + shrink + Bregman update, right-hand side, the
# system matrix K) are library kernels (include/nufft_mi355x.h, nufft_tv_*);
# A^H A is the plan's pair or its Toeplitz operator; CG's scalars stay on the
# device.
import ctypes  # noqa: E402

from . import _lib  # noqa: E402


def _p(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _s(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dims(x: torch.Tensor, batch_dims: int = 0):
    shape = tuple(x.shape[batch_dims:])
    return len(shape), (ctypes.c_int64 * len(shape))(*shape)


def tv_shrink(x: torch.Tensor, dd: torch.Tensor, bb: torch.Tensor, t: float):
    """For each axis a: z = grad_a x + b_a; d_a = shrink(z, t); b_a = z - d_a
    (dd, bb: [d, *x.shape], updated in place)."""
    d, n = _dims(x)
    with torch.cuda.device(x.device):
        _lib.call("nufft_tv_shrink", d, n, _p(x), _p(dd), _p(bb), ctypes.c_float(t), _s(x))


def tv_rhs(mu: float, ahy: torch.Tensor, lam: float, dd: torch.Tensor, bb: torch.Tensor, out: torch.Tensor,
           df: torch.Tensor | None = None, bf: torch.Tensor | None = None):
    """out = mu (ahy [+ df - bf]) + lam sum_a grad_a^T (d_a - b_a)."""
    d, n = _dims(ahy)
    with torch.cuda.device(ahy.device):
        _lib.call("nufft_tv_rhs", d, n, ctypes.c_float(mu), _p(ahy), None if df is None else _p(df),
                  None if bf is None else _p(bf), ctypes.c_float(lam), _p(dd), _p(bb), _p(out), _s(ahy))


def tv_normal(mu: float, ahax: torch.Tensor, lam: float, x: torch.Tensor, out: torch.Tensor):
    """out = mu ahax + lam sum_a grad_a^T grad_a x."""
    d, n = _dims(x)
    with torch.cuda.device(x.device):
        _lib.call("nufft_tv_normal", d, n, ctypes.c_float(mu), _p(ahax), ctypes.c_float(lam), _p(x), _p(out), _s(x))


def bregman_shrink(r: torch.Tensor, dv: torch.Tensor, bv: torch.Tensor, t: float):
    """z = r + b; d = shrink(z, t); b = z - d (elementwise, in place)."""
    with torch.cuda.device(r.device):
        _lib.call("nufft_bregman_shrink", ctypes.c_int64(r.numel()), _p(r), _p(dv), _p(bv), ctypes.c_float(t), _s(r))


def cg(apply, b: torch.Tensor, iters: int, x: torch.Tensor | None = None) -> torch.Tensor:
    """CG on a Hermitian positive semi-definite system, `iters` iterations
    from x (zero if None, updated in place otherwise); apply(v, out) writes
    the operator applied to v into out."""
    ap = torch.empty_like(b)
    if x is None:
        x = torch.zeros_like(b)
        r = b.clone()
    else:
        r = b - apply(x, ap)
    p = r.clone()
    rr = _dot_re(r, r)
    for _ in range(iters):
        apply(p, ap)
        alpha = rr / _dot_re(p, ap)
        x.add_(p * alpha)
        r.sub_(ap * alpha)
        rr_new = _dot_re(r, r)
        p.mul_(rr_new / rr).add_(r)
        rr = rr_new
    return x


def l1tv(plan: Plan, y: torch.Tensor, mu: float, lam: float, outer: int = 4, inner: int = 4, cg_iters: int = 15,
         lad: bool = False, normal=None) -> torch.Tensor:
    """L1TV-OLS (lad=False) or L1TV-LAD (lad=True) reconstruction with the
    split-Bregman iterations of the paper:
      K = mu A^H A + lam sum_a grad_a^T grad_a
      inner: rhs = mu (A^H y^k [+ d_f - b_f]) + lam sum_a grad_a^T (d_a - b_a)
             x = K^-1 rhs (cg_iters CG iterations from the current x)
             d_a = shrink(grad_a x + b_a, 1/lam), b_a += grad_a x - d_a
             LAD: r = A^H A x - A^H y, d_f = shrink(r + b_f, 1/mu), b_f += r - d_f
      outer: A^H y^{k+1} = A^H y^k + A^H y - A^H A x
    (the printed d_f update's b_y is read as b_f).  A^H A is applied as the
    pair, or by `normal` (e.g. plan.toeplitz()) when given."""
    N = plan.N
    d = len(N)
    dev = plan.device
    ybuf = torch.empty_like(y)

    def aha(v, out):
        if normal is not None:
            return normal(v, out=out)
        plan.forward(v, out=ybuf)
        return plan.adjoint(ybuf, out=out)

    ahy = plan.adjoint(y)
    ahyk = ahy.clone()
    x = torch.zeros(N, dtype=torch.complex64, device=dev)
    dd = torch.zeros((d,) + N, dtype=torch.complex64, device=dev)
    bb = torch.zeros_like(dd)
    df = torch.zeros(N, dtype=torch.complex64, device=dev) if lad else None
    bf = torch.zeros_like(df) if lad else None
    rhs = torch.empty_like(x)
    tmp = torch.empty_like(x)
    res = torch.empty_like(x)

    def kop(v, out):
        aha(v, tmp)
        tv_normal(mu, tmp, lam, v, out)
        return out

    for _ in range(outer):
        for _ in range(inner):
            tv_rhs(mu, ahyk, lam, dd, bb, rhs, df, bf)
            cg(kop, rhs, cg_iters, x)
            tv_shrink(x, dd, bb, 1.0 / lam)
            if lad:
                aha(x, res)
                res.sub_(ahy)
                bregman_shrink(res, df, bf, 1.0 / mu)
        aha(x, tmp)
        ahyk.add_(ahy).sub_(tmp)
    return x
