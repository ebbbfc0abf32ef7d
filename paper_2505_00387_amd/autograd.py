"""torch.autograd.Function around the HIP operator pair: forward = L, backward = L^T.

Because the library's adjoint is the exact transpose of its forward operator,
the gradient of any loss of d = L m with respect to m is L^T (dLoss/dd).
"""
from __future__ import annotations

import torch


class AAHRTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(m.contiguous())

    @staticmethod
    def backward(ctx, grad_d: torch.Tensor):
        return ctx.plan.adjoint(grad_d.contiguous()), None


def aahrt(m: torch.Tensor, plan) -> torch.Tensor:
    """Differentiable d = L m on the plan's batch (m: [batch, ntheta, nq, ntau] float32 on the GPU)."""
    return AAHRTFunction.apply(m, plan)
