"""Differentiable Joseph projector: torch.autograd.Functions over libdect.

The forward of JosephProjector is dect_project (A x); its backward is the
hand-written gather back-projector dect_backproject (A^T g), the exact
transpose of the forward matrix, so the gradient of any loss of A x is exact
up to FP32 rounding.  JosephBackprojector is the mirror pair.
"""
from __future__ import annotations

import torch

from . import configs as C
from . import dect


class JosephProjector(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, geom: C.Geometry):
        ctx.geom = geom
        return dect.project(x.contiguous(), geom)

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        return dect.backproject(gy.contiguous(), ctx.geom), None


class JosephBackprojector(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y: torch.Tensor, geom: C.Geometry):
        ctx.geom = geom
        return dect.backproject(y.contiguous(), geom)

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        return dect.project(gx.contiguous(), ctx.geom), None


def project(x: torch.Tensor, geom: C.Geometry) -> torch.Tensor:
    """A x for images [..., ny, nx], differentiable."""
    return JosephProjector.apply(x, geom)


def backproject(y: torch.Tensor, geom: C.Geometry) -> torch.Tensor:
    """A^T y for sinograms [..., V, B], differentiable."""
    return JosephBackprojector.apply(y, geom)
