"""torch.autograd.Function over the library: F(x, w) per restart (Def. 3)
with gradients with respect to the points x and the constraint weights w.

Forward runs ffsat_eval (objective, gradient, per-constraint values);
backward runs ffsat_vjp (gx = gF * grad, gw = sum_b gF_b WE_c(x_b)).  Torch
only carries the tensors.  The forward pass stores w as the problem's
weights (the problem is shared state of the plan).
"""
from __future__ import annotations

import torch

from .api import Plan


class FFSatObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, w: torch.Tensor, plan: Plan):
        if x.dtype != torch.float32 or w.dtype != torch.float32:
            raise TypeError("x and w must be float32")
        plan.problem.set_weights(w.detach().contiguous())
        need_x, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        out = plan.eval(x.detach().contiguous(), want_F=True, want_grad=need_x, want_con=need_w)
        ctx.plan = plan
        ctx.save_for_backward(out.get("grad"), out.get("con_val"))
        return out["F"]

    @staticmethod
    def backward(ctx, gF: torch.Tensor):
        grad, con_val = ctx.saved_tensors
        gx, gw = ctx.plan.vjp(gF.detach().contiguous().to(torch.float32), grad, con_val)
        return gx, gw, None


def objective(x: torch.Tensor, w: torch.Tensor, plan: Plan) -> torch.Tensor:
    """F[b] = sum_c w_c WE_c(x_b) for x [n][B], w [m]; differentiable in both."""
    return FFSatObjective.apply(x, w, plan)
