"""Unrolled ADM-TV with learnable per-step parameters (differentiable).

Each unrolled step k is one pass of the reconstruction procedure (Eq. 10)
with the BB step replaced by a learnable step alpha_k and learnable
(mu_k, rho_k, xi_k):
    z      = shrink(grad f - lambda / rho_k, 1 / rho_k)                (Eq. 8)
    G      = mu_k A^T (A f - g) + grad^T(rho_k (grad f - z) - lambda)   (Eq. 9)
    f     <- f - alpha_k G
    lambda <- lambda - xi_k (grad f - z)                                (Eq. 7)
Every step of it runs in libdect: A and A^T are the hand-written projector
pair, r = A f - g is dect_unrolled_residual, and the differences, the
shrinkage, G and both updates are dect_unrolled_step, whose backward is the
hand-written dect_unrolled_step_backward.  Torch only records the graph and
holds the tensors.  Activations are checkpointed every `checkpoint_every`
steps.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import torch
from torch.utils.checkpoint import checkpoint

from . import autograd as AG
from . import configs as C
from . import dect


class _Residual(torch.autograd.Function):
    """r = p - g (g is data: it gets no gradient)."""

    @staticmethod
    def forward(ctx, p, g):
        return dect.unrolled_residual(p.contiguous(), g.contiguous())

    @staticmethod
    def backward(ctx, gr):
        return gr, None


class _Step(torch.autograd.Function):
    """(f, lambda_x, lambda_y, hb = A^T r, (mu, rho, xi, alpha)) -> (f', lambda')."""

    @staticmethod
    def forward(ctx, f, lx, ly, hb, params):
        f, lx, ly, hb = (t.contiguous() for t in (f, lx, ly, hb))
        params = params.contiguous()
        ctx.save_for_backward(f, lx, ly, hb, params)
        return dect.unrolled_step(f, lx, ly, hb, params)

    @staticmethod
    def backward(ctx, gfo, glxo, glyo):
        f, lx, ly, hb, params = ctx.saved_tensors
        cot = [torch.zeros_like(f) if t is None else t.contiguous() for t in (gfo, glxo, glyo)]
        gf, glx, gly, ghb, gp = dect.unrolled_step_backward(f, lx, ly, hb, params, *cot)
        return gf, glx, gly, ghb, gp


def adm_step(f, lx, ly, g, geom: C.Geometry, mu, rho, xi, alpha):
    """One unrolled ADM-TV step for a batch f [B, ny, nx], g [B, V, bins];
    mu, rho, xi, alpha: 0-d float32 device tensors."""
    r = _Residual.apply(AG.project(f, geom), g)
    hb = AG.backproject(r, geom)
    params = torch.stack((mu, rho, xi, alpha))
    return _Step.apply(f, lx, ly, hb, params)


class UnrolledADM(torch.nn.Module):
    """K unrolled ADM-TV steps with learnable positive (mu_k, rho_k, xi_k, alpha_k)."""

    def __init__(self, geom: C.Geometry, n_steps: int = 10, mu: float = 0.25,
                 rho: float = 1024.0, xi: float = 256.0,
                 alphas: Optional[Sequence[float]] = None, checkpoint_every: int = 2):
        super().__init__()
        self.geom = geom
        self.n_steps = n_steps
        self.checkpoint_every = checkpoint_every
        if alphas is None:
            alphas = [1e-4] * n_steps
        self.log_mu = torch.nn.Parameter(torch.full((n_steps,), math.log(mu), dtype=torch.float64))
        self.log_rho = torch.nn.Parameter(torch.full((n_steps,), math.log(rho), dtype=torch.float64))
        self.log_xi = torch.nn.Parameter(torch.full((n_steps,), math.log(xi), dtype=torch.float64))
        self.log_alpha = torch.nn.Parameter(torch.log(torch.tensor(list(alphas), dtype=torch.float64)))

    def params_of(self, k: int):
        return (torch.exp(self.log_mu[k]).float(), torch.exp(self.log_rho[k]).float(),
                torch.exp(self.log_xi[k]).float(), torch.exp(self.log_alpha[k]).float())

    def _segment(self, k0: int, k1: int, g):
        def run(f, lx, ly, *params):
            for j, k in enumerate(range(k0, k1)):
                mu, rho, xi, alpha = params[4 * j:4 * j + 4]
                f, lx, ly = adm_step(f, lx, ly, g, self.geom, mu, rho, xi, alpha)
            return f, lx, ly
        return run

    def forward(self, g: torch.Tensor, f0: Optional[torch.Tensor] = None,
                use_checkpoint: bool = True):
        """g: [B, V, bins] (already beta-scaled).  Returns f after K steps."""
        B = g.shape[0]
        ny, nx = self.geom.ny, self.geom.nx
        f = torch.zeros((B, ny, nx), device=g.device) if f0 is None else f0
        lx = torch.zeros_like(f)
        ly = torch.zeros_like(f)
        step = max(1, self.checkpoint_every)
        for k0 in range(0, self.n_steps, step):
            k1 = min(self.n_steps, k0 + step)
            params = []
            for k in range(k0, k1):
                params.extend(self.params_of(k))
            fn = self._segment(k0, k1, g)
            if use_checkpoint and torch.is_grad_enabled():
                f, lx, ly = checkpoint(fn, f, lx, ly, *params, use_reentrant=False)
            else:
                f, lx, ly = fn(f, lx, ly, *params)
        return f
