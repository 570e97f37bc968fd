"""torch.autograd bindings of the dedispersion sum with learnable per-tap weights.

DedisperseFn: y = A_w x (all trials, all outputs); backward runs the library's
adjoint kernels (gradient with respect to the weights in fp64, and optionally the
input).  GatherFn: only the outputs y[b_e, d_e, t_e] (a matched filter evaluated
at known pulse positions); its backward is the sparse adjoint, whose cost does not
grow with the number of trials or outputs.
"""
from __future__ import annotations

import torch

from .api import Plan


class DedisperseFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, w: torch.Tensor, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(x, w)
        return plan.dedisperse(x, weights=w.detach())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        x, w = ctx.saved_tensors
        plan = ctx.plan
        gx, gw = plan.backward(gy, x, need_x=ctx.needs_input_grad[0],
                               need_w=ctx.needs_input_grad[1], weights=w.detach())
        gwt = gw.to(w.dtype) if gw is not None else None
        return gx, gwt, None


class GatherFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, w: torch.Tensor, plan: Plan, b, d, t):
        ctx.plan = plan
        ctx.idx = (b, d, t)
        ctx.save_for_backward(x, w)
        return plan.gather(x, b, d, t, weights=w.detach())

    @staticmethod
    def backward(ctx, gv: torch.Tensor):
        x, w = ctx.saved_tensors
        b, d, t = ctx.idx
        gw = ctx.plan.backward_sparse(x, b, d, t, gv.contiguous())
        return None, gw.to(w.dtype), None, None, None, None


def matched_filter_loss(x: torch.Tensor, w: torch.Tensor, plan: Plan, b, d, t, sigma: float = 1.0,
                        sparse: bool = True) -> torch.Tensor:
    """Negative mean S/N of the weighted sum at known pulse positions:
    L = -(1/B) sum_e y[b_e, d_e, t_e] / (sigma * ||w||), the noise standard deviation
    of one weighted output being sigma * ||w|| for independent unit-variance samples."""
    if sparse:
        v = GatherFn.apply(x, w, plan, b, d, t)
    else:
        y = DedisperseFn.apply(x, w, plan)
        bi = torch.as_tensor(b, device=x.device, dtype=torch.long)
        di = torch.as_tensor(d, device=x.device, dtype=torch.long)
        ti = torch.as_tensor(t, device=x.device, dtype=torch.long)
        v = y[bi, di, ti]
    # normalise in fp64: the two gradient terms of the quotient nearly cancel
    norm = torch.linalg.vector_norm(w.double())
    return -(v.double() / (sigma * norm)).mean()
