"""Differentiable projector: forward = A x (HIP forward projection), backward = A^T g
(HIP matched back projection, the exact transpose of the forward lengths).

The forward model of Sec. I (y = A x + e) as a torch.autograd.Function, so that any
loss built from A x (for example 1/2 ||y - A x||^2 plus a TV term written in torch)
differentiates through the on-the-fly projectors.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from .bsgd import Geometry


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, geom: Geometry, views: Optional[Sequence[int]], block: int):
        ctx.geom, ctx.views, ctx.block = geom, views, block
        return geom.forward_project(x.detach().contiguous(), views=views, block=block)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        gx = ctx.geom.back_project(grad_y.detach().contiguous(), views=ctx.views, block=ctx.block)
        return gx, None, None, None


def project(x: torch.Tensor, geom: Geometry, views: Optional[Sequence[int]] = None, block: int = -1):
    """A_{views}^{J} x as a differentiable op (x: flat FP32 device tensor)."""
    if x.dtype != torch.float32 or not x.is_cuda:
        raise TypeError("project expects a float32 device tensor")
    return _Project.apply(x, geom, views, block)


def tv_smooth(x: torch.Tensor, shape, eps: float = 1e-8) -> torch.Tensor:
    """Isotropic TV with backward differences (zero across the low boundary), smoothed
    by eps inside the square root so it is differentiable (plain torch ops)."""
    v = x.view(*shape)
    sq = torch.zeros_like(v)
    for a in range(v.dim()):
        d = torch.diff(v, dim=a)
        pad = [0, 0] * v.dim()
        pad[2 * (v.dim() - 1 - a)] = 1  # one zero difference at the low boundary
        sq = sq + torch.nn.functional.pad(d, pad) ** 2
    return torch.sqrt(sq + eps).sum()
