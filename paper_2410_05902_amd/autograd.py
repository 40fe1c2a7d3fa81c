"""torch.autograd face of the differentiation form.

``batch_objective(model, xb, sigma)`` is the batch objective of Section 3,
f(xb, sigma) = (1/b) sum_x min_j ||phi_sigma(x) - C_j||^2, for the Gaussian
kernel in bandwidth form exp(-||x-y||^2 / (2 sigma^2)), with the model's
current centers (support points and weights) held constant.  Forward and
backward run in libmbkk (mbkk_objective_fwd / mbkk_objective_bwd); the
backward recomputes kernel values instead of storing them.  Gradients flow to
the batch coordinates xb and to sigma (a 0-dim tensor), e.g. for tuning the
bandwidth by gradient steps.
"""
from __future__ import annotations

import torch


class BatchObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xb: torch.Tensor, sigma: torch.Tensor, model):
        s = float(sigma.detach())
        f, labels = model.objective_fwd(xb.detach(), s)
        ctx.model = model
        ctx.sigma = s
        ctx.sig_meta = (sigma.dtype, sigma.device)
        ctx.save_for_backward(xb.detach(), labels)
        return torch.tensor(f, dtype=torch.float64, device=xb.device)

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        xb, labels = ctx.saved_tensors
        g = float(grad_f)
        dX, ds = ctx.model.objective_bwd(xb, ctx.sigma, labels, g)
        dsig = None
        if ctx.needs_input_grad[1]:
            dsig = torch.tensor(ds, dtype=ctx.sig_meta[0], device=ctx.sig_meta[1])
        return (dX if ctx.needs_input_grad[0] else None), dsig, None


def batch_objective(model, xb: torch.Tensor, sigma: torch.Tensor) -> torch.Tensor:
    """f(xb, sigma) as a differentiable scalar (float64)."""
    if not torch.is_tensor(sigma):
        sigma = torch.tensor(float(sigma), dtype=torch.float64)
    return BatchObjective.apply(xb, sigma, model)
