"""torch.autograd.Function over the library's hand-written adjoint.

``log_posterior(heights, problem)`` returns the per-chain log posterior of a
[n_chains, S-1, R, C] height tensor; its backward hands back the gradient the
adjoint kernels computed in the forward call (scaled by the incoming
gradient), so torch optimisers and samplers can drive the surfaces directly.
"""
from __future__ import annotations

import torch


class LogPosterior(torch.autograd.Function):
    @staticmethod
    def forward(ctx, heights, problem):
        h = heights.detach()
        if not h.is_contiguous():
            h = h.contiguous()
        lp, grad = problem.logpost_grad_batch(h)
        ctx.save_for_backward(grad)
        ctx.n_free = problem.S - 1
        return lp

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        scale = grad_out.to(grad.dtype).view(-1, 1, 1, 1)
        return grad[:, : ctx.n_free] * scale, None


def log_posterior(heights: torch.Tensor, problem) -> torch.Tensor:
    """Differentiable log posterior (float64 per chain) of the free surfaces."""
    return LogPosterior.apply(heights, problem)
