"""Unrolled ADM-TV with learnable per-step parameters (differentiable).

Each unrolled step k is one pass of the reconstruction procedure (Eq. 10)
with the BB step replaced by a learnable step alpha_k and learnable
(mu_k, rho_k, xi_k):
    z      = shrink(grad f - lambda / rho_k, 1 / rho_k)                (Eq. 8)
    G      = mu_k A^T (A f - g) + grad^T(rho_k (grad f - z) - lambda)   (Eq. 9)
    f     <- f - alpha_k G
    lambda <- lambda - xi_k (grad f - z)                                (Eq. 7)
A and A^T are the hand-written projector pair (autograd-aware); the
finite differences and shrinkage are elementwise torch ops on the device.
Activations are checkpointed every `checkpoint_every` steps.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import torch
from torch.utils.checkpoint import checkpoint

from . import autograd as AG
from . import configs as C


def grad2d(x: torch.Tensor):
    """Backward differences of Eq. 2 (zero on the first column/row)."""
    gx = torch.zeros_like(x)
    gy = torch.zeros_like(x)
    gx[..., :, 1:] = x[..., :, 1:] - x[..., :, :-1]
    gy[..., 1:, :] = x[..., 1:, :] - x[..., :-1, :]
    return gx, gy


def grad2d_T(px: torch.Tensor, py: torch.Tensor) -> torch.Tensor:
    """Exact adjoint of grad2d."""
    out = torch.zeros_like(px)
    out[..., :, 1:] += px[..., :, 1:]
    out[..., :, :-1] -= px[..., :, 1:]
    out[..., 1:, :] += py[..., 1:, :]
    out[..., :-1, :] -= py[..., 1:, :]
    return out


def shrink(vx: torch.Tensor, vy: torch.Tensor, t: torch.Tensor):
    """Isotropic shrinkage max(|v| - t, 0) v / |v| (zero where |v| <= t).

    |v| is evaluated as sqrt(max(|v|^2, 1e-30)): identical for |v| > 1e-15 (far
    below any threshold t), and finite in value and gradient at v = 0.
    """
    n = torch.sqrt(torch.clamp(vx * vx + vy * vy, min=1e-30))
    s = torch.clamp(n - t, min=0.0) / n
    return s * vx, s * vy


def adm_step(f, lx, ly, g, geom: C.Geometry, mu, rho, xi, alpha):
    """One unrolled ADM-TV step for a batch f [B, ny, nx], g [B, V, bins]."""
    r = AG.project(f, geom) - g
    h = mu * AG.backproject(r, geom)
    dx, dy = grad2d(f)
    zx, zy = shrink(dx - lx / rho, dy - ly / rho, 1.0 / rho)
    G = h + grad2d_T(rho * (dx - zx) - lx, rho * (dy - zy) - ly)
    f = f - alpha * G
    nx_, ny_ = grad2d(f)
    lx = lx - xi * (nx_ - zx)
    ly = ly - xi * (ny_ - zy)
    return f, lx, ly


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
