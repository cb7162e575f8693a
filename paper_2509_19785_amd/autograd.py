"""The tsNET cost as a torch.autograd.Function.

Forward evaluates C = C_KL + C_CMP + C_ENT (Eq. 1, the entropy term in the
kernel form whose gradient is Eq. 8) with ``tsnet_cost``; backward is the
hand-written gradient kernel ``tsnet_grad`` scaled by the incoming gradient.
Both run the FP32 interpolation path, so any torch optimiser can drive the
layout. With a batch of graphs the forward returns the sum of the per-graph
costs (each graph's gradient is independent of the others).
"""
from __future__ import annotations

import torch

from .api import Params, Problem


class TsnetCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X: torch.Tensor, problem: Problem, params: Params):
        Xd = X.detach()
        cost = problem.cost(Xd, params)            # [graphs][KL, CMP, ENT, total], FP64
        ctx.problem = problem
        ctx.params = params
        ctx.save_for_backward(Xd)
        return cost[:, 3].sum()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (Xd,) = ctx.saved_tensors
        G, _ = ctx.problem.grad(Xd, ctx.params)
        return G * grad_out.to(G.dtype), None, None


def tsnet_cost(X: torch.Tensor, problem: Problem, params: Params | None = None) -> torch.Tensor:
    """Differentiable cost of layout X (float32 [n, 2] on the problem's device)."""
    return TsnetCost.apply(X, problem, params or Params())
