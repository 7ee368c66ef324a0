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
