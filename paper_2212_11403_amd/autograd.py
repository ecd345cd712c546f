"""torch.autograd.Functions for the PAC log-likelihood and the recombination
map.

PACLoglik forward: sum over recipients of log P(h_i | h_-i) (forward sweeps
only); backward: the gradient with respect to every rho_l and mu from the
library's checkpointed adjoint (ls_loglik_grad), scaled by the incoming
gradient.

RhoMap forward: rho = 1 - exp(-s (cM / 100)^gamma) (eq. rho, ls_calc_rho);
backward: the chain rule to s and gamma (ls_rho_map_grad). Composed,
PACLoglik.apply(RhoMap.apply(cM, s, gamma), mu, ...) differentiates the PAC
with respect to the map parameters.
"""

from __future__ import annotations

import torch

from . import api


class PACLoglik(torch.autograd.Function):
    """PACLoglik.apply(rho, mu, H, N, prec="fp32", recipients=None) -> scalar.

    rho: float64 device tensor [L-1]; mu: float64 0-d tensor, or [L] (one
    per variant); H: packed haplotypes (device int32 [L][stride] or numpy
    uint32).
    """

    @staticmethod
    def forward(ctx, rho, mu, H, N, prec="fp32", recipients=None):
        mu_arg = float(mu) if mu.dim() == 0 else mu.detach().to(torch.float64)
        model = api.Model(H, int(N), rho.detach().to(torch.float64), mu_arg)
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


class RhoMap(torch.autograd.Function):
    """RhoMap.apply(cM, s, gamma) -> rho [n]. cM: float64 [n] (centimorgans,
    not differentiated); s, gamma: float64 0-d tensors."""

    @staticmethod
    def forward(ctx, cM, s, gamma):
        c = cM.detach().to(torch.float64)
        sv, gv = float(s), float(gamma)
        ctx.save_for_backward(c)
        ctx.sg = (sv, gv, s.shape, gamma.shape)
        return api.calc_rho(c, sv, gv)

    @staticmethod
    def backward(ctx, g):
        (c,) = ctx.saved_tensors
        sv, gv, s_shape, g_shape = ctx.sg
        out = api.rho_map_grad(c, sv, gv, g.detach().to(torch.float64).contiguous())
        return None, out[0].reshape(s_shape), out[1].reshape(g_shape)
