"""torch.autograd support for the NUFFT pair.

The forward is y = A(om) x (paper Section 2.1, Eq. A = VFS; coil mode y_i =
A(c_i x), Section 2.2).  The backward is written by hand, with torch's
convention for complex tensors (grad = dL/dRe + i dL/dIm):
  - image:      grad_x  = A^H grad_y   (sum_i conj(c_i) A^H grad_y_i with coils),
                the adjoint of Section 2.1;
  - trajectory: grad_om[m, a] = sum_i Re(conj(grad_y_i[m]) dy_i[m]/dom[m, a]),
                through the derivative of the interpolation kernel
                (nufft_grad_points).
Both run in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from .plan import Plan


class NufftFunction(torch.autograd.Function):
    """y = A(om) x for one image ([*N]) or a batch ([B, *N]) on `plan`.

    `om` must be the trajectory the plan currently holds (NufftOp keeps them in
    step); it is an input only so autograd can route its gradient.  The
    backward runs on the plan's trajectory; if the plan was re-binned
    (Plan.set_points) between this forward and its backward, the backward
    raises instead of returning gradients for the wrong trajectory."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, om: torch.Tensor, plan: Plan):
        x = x.contiguous()
        batched = x.dim() == len(plan.N) + 1
        y = plan.forward_batched(x) if batched else plan.forward(x)
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.batched = batched
        ctx.save_for_backward(x)
        return y

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        (x,) = ctx.saved_tensors
        plan: Plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("the NUFFT plan was re-binned for another trajectory (set_points) between this "
                               "forward and its backward; run backward before changing the trajectory")
        gy = gy.contiguous()
        gx = gom = None
        if ctx.needs_input_grad[0]:
            gx = plan.adjoint_batched(gy) if ctx.batched else plan.adjoint(gy)
        if ctx.needs_input_grad[1]:
            if ctx.batched:
                gom = plan.grad_points_batched(x, gy)
            else:
                gom = plan.grad_points(x, gy)
        return gx, gom, None


class NufftOp(torch.nn.Module):
    """Differentiable NUFFT with a plan that follows the trajectory.

    op = NufftOp(om, N, K, J, coils=None); y = op(x) or y = op(x, om).  When a
    trajectory tensor is passed and its storage or version changed since the
    last call, the plan is re-binned for it (nufft_set_points) before the
    transform."""

    def __init__(self, om: torch.Tensor, N, K=None, J: int = 6, coils: torch.Tensor | None = None):
        super().__init__()
        self.plan = Plan(om.detach().contiguous(), N, K, J, coils=coils)
        self._om_key = self._key(om)

    @staticmethod
    def _key(om):
        return (om.data_ptr(), om._version)

    def forward(self, x: torch.Tensor, om: torch.Tensor | None = None) -> torch.Tensor:
        if om is None:
            om = torch.empty((self.plan.M, self.plan.d), dtype=torch.float32, device=x.device)
            return NufftFunction.apply(x, om, self.plan)
        key = self._key(om)
        if key != self._om_key:
            self.plan.set_points(om.detach().contiguous())
            self._om_key = key
        return NufftFunction.apply(x, om, self.plan)

    def adjoint(self, y: torch.Tensor) -> torch.Tensor:
        batched = y.dim() == (2 if self.plan.C else 1) + 1
        return self.plan.adjoint_batched(y.contiguous()) if batched else self.plan.adjoint(y.contiguous())


def nufft(x: torch.Tensor, om: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Functional form: y = A(om) x on `plan` (which must hold `om`)."""
    return NufftFunction.apply(x, om, plan)
