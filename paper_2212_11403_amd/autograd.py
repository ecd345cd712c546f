"""torch.autograd.Function for the PAC log-likelihood.

forward: sum over recipients of log P(h_i | h_-i) (forward sweeps only).
backward: the gradient with respect to every rho_l and mu from the library's
checkpointed adjoint (ls_loglik_grad), scaled by the incoming gradient.
"""

from __future__ import annotations

import torch

from . import api


class PACLoglik(torch.autograd.Function):
    """PACLoglik.apply(rho, mu, H, N, prec="fp32", recipients=None) -> scalar.

    rho: float64 device tensor [L-1]; mu: float64 0-d tensor; H: packed
    haplotypes (device int32 [L][stride] or numpy uint32).
    """

    @staticmethod
    def forward(ctx, rho, mu, H, N, prec="fp32", recipients=None):
        model = api.Model(H, int(N), rho.detach().to(torch.float64), float(mu))
        out = api.loglik_grad(model, recipients, prec, grad=False)
        ctx.model = model
        ctx.prec = prec
        ctx.recipients = recipients
        ctx.mu_shape = mu.shape
        return out["pac"].reshape(())

    @staticmethod
    def backward(ctx, g):
        out = api.loglik_grad(ctx.model, ctx.recipients, ctx.prec, grad=True)
        g_rho = g * out["grad_rho"]
        g_mu = (g * out["grad_mu"]).reshape(ctx.mu_shape)
        return g_rho, g_mu, None, None, None, None
