"""torch.autograd bridge for the differentiation form.

``objective(q, mu, spec, n_draws)`` returns the Monte Carlo objective at the
continuous design points q [B, d] for prior means mu = (mu_b0, mu_b1); its
backward pass uses the library's adjoint kernel (bmd_grad_design), which
regenerates the draws from their Philox counters.
"""
from __future__ import annotations

import torch

from . import Problem


class BmdObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, mu, spec, n_draws, precision):
        s = dict(spec)
        s["mu_b0"], s["mu_b1"] = (float(x) for x in mu.detach().cpu().tolist())
        with Problem(s) as p:
            obj, gq, gmu = p.grad_design(q.detach(), n_draws, precision, want_grad=True)
        ctx.save_for_backward(gq, gmu)
        return obj.to(q.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        gq, gmu = ctx.saved_tensors
        g = grad_out.to(torch.float64)
        grad_q = (g[:, None] * gq)
        grad_mu = (g[:, None] * gmu).sum(0)
        return grad_q, grad_mu, None, None, None


def objective(q, mu, spec, n_draws, precision="fp32"):
    return BmdObjective.apply(q, mu, spec, n_draws, precision)
