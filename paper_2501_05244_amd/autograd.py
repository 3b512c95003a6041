"""torch.autograd.Function over the C-ABI forward and hand-written adjoint.

    V = nursd(P, relay_xy, plan)      # complex64 [Z][ny][nx]

The backward calls nursd_adjoint, which recomputes every per-frequency
quantity (no forward state is kept besides P and the positions): it returns
the gradient with respect to the complex phasors P and, when relay_xy
requires grad, with respect to the relay positions.

The plan holds one set of relay positions at a time.  Each forward binds
the positions it was given, and each backward binds the positions saved by
its own forward; a plan that already holds that very tensor at its current
version is not re-binned.  Interleaved forwards with different positions
are therefore each differentiated at their own positions, and autograd's
saved-tensor version check rejects positions changed in place between a
forward and its backward.
"""
from __future__ import annotations

import torch

from .api import Plan


class NURSDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P: torch.Tensor, relay_xy: torch.Tensor, plan: Plan):
        plan.bind_points(relay_xy)
        V, _ = plan.forward_phasor(P.detach().contiguous(), intensity=False)
        ctx.save_for_backward(P, relay_xy)
        ctx.plan = plan
        return V

    @staticmethod
    def backward(ctx, gV: torch.Tensor):
        P, relay_xy = ctx.saved_tensors
        ctx.plan.bind_points(relay_xy)
        want_xy = ctx.needs_input_grad[1]
        gP, gxy = ctx.plan.adjoint(gV.contiguous(), P.detach().contiguous() if want_xy else None)
        return (gP if ctx.needs_input_grad[0] else None), (gxy if want_xy else None), None


def nursd(P: torch.Tensor, relay_xy: torch.Tensor, plan: Plan) -> torch.Tensor:
    return NURSDFunction.apply(P, relay_xy, plan)
