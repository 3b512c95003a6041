"""torch.autograd.Function over the C-ABI forward and hand-written adjoint.

    V = nursd(P, relay_xy, plan)      # complex64 [Z][ny][nx]

The backward calls nursd_adjoint, which recomputes every per-frequency
quantity (no forward state is kept besides P and the positions): it returns
the gradient with respect to the complex phasors P and, when relay_xy
requires grad, with respect to the relay positions.
"""
from __future__ import annotations

import torch

from .api import Plan


class NURSDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P: torch.Tensor, relay_xy: torch.Tensor, plan: Plan):
        key = (relay_xy.data_ptr(), relay_xy._version)
        if getattr(plan, "_points_key", None) != key:
            plan.set_points(relay_xy.detach().contiguous())
            plan._points_key = key
        V, _ = plan.forward_phasor(P.detach().contiguous(), intensity=False)
        ctx.save_for_backward(P, relay_xy)
        ctx.plan = plan
        return V

    @staticmethod
    def backward(ctx, gV: torch.Tensor):
        P, relay_xy = ctx.saved_tensors
        want_xy = ctx.needs_input_grad[1]
        gP, gxy = ctx.plan.adjoint(gV.contiguous(), P.detach().contiguous() if want_xy else None)
        return (gP if ctx.needs_input_grad[0] else None), (gxy if want_xy else None), None


def nursd(P: torch.Tensor, relay_xy: torch.Tensor, plan: Plan) -> torch.Tensor:
    return NURSDFunction.apply(P, relay_xy, plan)
