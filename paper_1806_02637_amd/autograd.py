"""The consistency cost as a differentiable torch function.

Forward calls ecc_cost (or ecc_cost_grad when theta requires grad, keeping
the gradient the adjoint kernel produced); backward scales that gradient by
the incoming d loss / d cost.  The engine does all the arithmetic.
"""
from __future__ import annotations

import math

import torch


class EccCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, scan, K, R_mm, c, geom, kappa):
        if theta.requires_grad:
            cost, grad = scan.cost_grad(theta.detach(), K, R_mm, c=c, geom=geom, kappa=kappa)
            ctx.save_for_backward(grad)
        else:
            cost = scan.cost(theta, K, R_mm, c=c, geom=geom, kappa=kappa)
        return cost

    @staticmethod
    def backward(ctx, grad_cost):
        (grad,) = ctx.saved_tensors
        g = grad_cost.to(torch.float64)[:, None, None] * grad.to(torch.float64)
        return g, None, None, None, None, None, None


def ecc_cost(theta: torch.Tensor, scan, K: int, R_mm: float, c: float = math.inf, geom: str = "f32",
             kappa: str = "object"):
    """cost[B] = sum over view pairs of the robust pairwise inconsistency for
    motion hypotheses theta [B, N, 6] (FP64, device); kappa selects the
    sampled plane range ("object" sphere or "detector"-bounded)."""
    return EccCost.apply(theta, scan, K, R_mm, c, geom, kappa)
