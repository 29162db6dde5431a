"""torch.autograd.Function over afq_energy / afq_energy_backward.

LocalEnergy.apply(h1, chol, W, weights, phi_t, n_up, n_dn, e_core=0.0,
precision="fp64") returns the weighted mixed energy
    Ebar = sum_w w_w Re E_L(W_w) / sum_w w_w
as a 0-dim float64 tensor on the GPU. Its backward gives dEbar/dh1,
dEbar/dchol (every entry, not symmetrised) and dEbar/dW in torch's complex
convention (d/dRe + i d/dIm); the trial and the weights are held fixed. The
library recomputes Theta and Omega in the backward call instead of keeping
them from the forward call.
"""
from __future__ import annotations

import torch

from . import api


class LocalEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h1, chol, W, weights, phi_t, n_up, n_dn, e_core=0.0, precision="fp64"):
        sysg = api.System(h1.detach(), chol.detach(), phi_t.detach(), n_up, n_dn, e_core, precision)
        wk = api.Walkers(sysg, W.shape[0], W.detach(), weights.detach())
        _, _, _, emix = wk.energy()
        ctx.sysg, ctx.wk = sysg, wk
        return emix[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        scale = float(grad_out)
        d_h1, d_chol, d_w = api.energy_backward(ctx.sysg, ctx.wk, scale)
        ctx.wk.close()
        ctx.sysg.close()
        return d_h1, d_chol, d_w, None, None, None, None, None, None
