"""torch.autograd.Functions for the PAC log-likelihood and the recombination
map.

PACLoglik forward: sum over recipients of log P(h_i | h_-i) from the
checkpointing forward sweep; backward: the gradient with respect to every
rho_l and mu from the library's adjoint over those checkpoints, scaled by
the incoming gradient.

RhoMap forward: rho = 1 - exp(-s (cM / 100)^gamma) (eq. rho, ls_calc_rho);
backward: the chain rule to s and gamma (ls_rho_map_grad). Composed,
PACLoglik.apply(RhoMap.apply(cM, s, gamma), mu, ...) differentiates the PAC
with respect to the map parameters.
"""

from __future__ import annotations

import torch

from . import api


# The model of the last PACLoglik.apply, reused while the haplotypes stay the
# same device tensor (same storage, shape and version): only the parameters
# are set again (ls_model_init in the existing workspace), so repeated
# evaluations in an optimisation loop neither upload H nor allocate.
_MODEL_CACHE = {}


def _model_for(H, N, rho, mu):
    rho = rho.detach().to(torch.float64)
    mu_arg = float(mu) if mu.dim() == 0 else mu.detach().to(torch.float64)
    if torch.is_tensor(H) and H.is_cuda:
        key = (H.data_ptr(), tuple(H.shape), H._version, int(N), H.device)
        m = _MODEL_CACHE.get("model")
        if m is not None and _MODEL_CACHE.get("key") == key:
            m.update(rho, mu_arg)
            return m
        m = api.Model(H, int(N), rho, mu_arg, device=H.device)
        _MODEL_CACHE.clear()
        _MODEL_CACHE.update(key=key, model=m)
        return m
    return api.Model(H, int(N), rho, mu_arg)


class PACLoglik(torch.autograd.Function):
    """PACLoglik.apply(rho, mu, H, N, prec="fp32", recipients=None) -> scalar.

    rho: float64 device tensor [L-1]; mu: float64 0-d tensor, or [L] (one
    per variant); H: packed haplotypes (device int32 [L][stride] or numpy
    uint32). The forward runs the checkpointing forward sweep
    (ls_loglik_checkpoint) and keeps its checkpoints; the backward runs only
    the recompute and adjoint passes over them (ls_loglik_grad_adjoint), so
    a forward plus backward costs one gradient, and both give the same bits
    as ls_loglik_grad. With H a device tensor the model is reused across
    applies while H is unchanged.
    """

    @staticmethod
    def forward(ctx, rho, mu, H, N, prec="fp32", recipients=None):
        model = _model_for(H, N, rho, mu)
        ck = api.Checkpoints(model, recipients, prec)
        ctx.ck = ck
        ctx.mu_shape = mu.shape
        return ck.pac.reshape(())

    @staticmethod
    def backward(ctx, g):
        g_rho, g_mu = ctx.ck.gradient()
        ctx.ck = None
        return g * g_rho, (g * g_mu).reshape(ctx.mu_shape), None, None, None, None


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
