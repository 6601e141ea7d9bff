"""torch.autograd wrapper of the likelihood: forward smc_loglik, backward
smc_loglik_backward (the hand-written adjoint).  Marshalling only."""
from __future__ import annotations

import torch

from . import _lib


class SmcLoglik(torch.autograd.Function):
    """loglik[p] = log p(y_{1:t} | theta[:, p]) for theta of shape [d, P]
    (FP64, on the model's device)."""

    @staticmethod
    def forward(ctx, theta, model, t):
        theta = theta.contiguous()
        ctx.model, ctx.t = model, t
        ctx.save_for_backward(theta)
        return _lib.smc_loglik(model, theta, t)

    @staticmethod
    def backward(ctx, grad_out):
        (theta,) = ctx.saved_tensors
        dtheta = _lib.smc_loglik_backward(ctx.model, theta, ctx.t,
                                          grad_out.contiguous().to(torch.float64))
        return dtheta, None, None


def loglik(theta, model, t):
    return SmcLoglik.apply(theta, model, t)
