"""Omega as a differentiable torch function.

`OmegaFn` wraps the library's gradient sweep (omega_grad): the forward pass
returns Omega_eps(Delta, Q) per point and band (Eq. (5)), and the saved
derivatives dOmega/dDelta, dOmega/dQ and dOmega/dmu (from differentiating
Eq. (4)-(5) by hand) serve the backward pass.  All arithmetic runs in the
library's kernels.
"""
from __future__ import annotations

import torch

from . import api


class OmegaFn(torch.autograd.Function):
    """Omega[p, b] at delta[p, b], q[p, b, :] with chemical potential mu.

    Inputs: delta [n_pts, nb] and q [n_pts, nb, 2] float64 CUDA tensors, mu a
    0-d float64 tensor; non-tensor arguments: model dict (its mu is replaced),
    host point list, band mask, optional workspace tensor."""

    @staticmethod
    def forward(ctx, delta, q, mu, model, pts, bands, workspace):
        m = dict(model)
        m["mu"] = float(mu)
        om, gd, gq, gm = api.grad(m, pts, delta.detach(), q.detach(), bands,
                                  device=delta.device, workspace=workspace)
        ctx.save_for_backward(gd, gq, gm)
        ctx.mu_shape = mu.shape
        return om

    @staticmethod
    def backward(ctx, g):
        gd, gq, gm = ctx.saved_tensors
        grad_delta = g * gd if ctx.needs_input_grad[0] else None
        grad_q = g.unsqueeze(-1) * gq if ctx.needs_input_grad[1] else None
        grad_mu = (g * gm).sum().reshape(ctx.mu_shape) if ctx.needs_input_grad[2] else None
        return grad_delta, grad_q, grad_mu, None, None, None, None


def omega(model, pts, delta, q, mu=None, bands: int = api.OMEGA_BAND_BOTH, workspace=None):
    """Differentiable Omega; mu defaults to the model's (as a tensor without grad)."""
    if mu is None:
        mu = torch.tensor(float(model["mu"]), dtype=torch.float64, device=delta.device)
    return OmegaFn.apply(delta, q, mu, model, pts, bands, workspace)
