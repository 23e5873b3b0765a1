"""Differentiable subset projector: forward y = A_i x, backward grad_x = A_i^T grad_y.

The backward pass is the library's backprojector, which is the exact adjoint of the projector
(same fixed-point ray walk and interpolation weights), so the gradient of any loss of y is
correct without autograd tracing through the projector.  Slices of x ([nz][ny][nx]) are
independent images, e.g. a batch.
"""
from __future__ import annotations

import torch

from . import api


class ProjectSubset(torch.autograd.Function):
    """``ProjectSubset.apply(x, geom, subset=-1)`` -> y with shape geom.sino_shape(subset)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, geom: "api.Geometry", subset: int = -1):
        ctx.geom = geom
        ctx.subset = int(subset)
        return api.project(geom, x.detach().contiguous(), ctx.subset)

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        grad_x = None
        if ctx.needs_input_grad[0]:
            grad_x = api.backproject(ctx.geom, grad_y.contiguous(), ctx.subset)
        return grad_x, None, None


def project_subset(x: torch.Tensor, geom: "api.Geometry", subset: int = -1) -> torch.Tensor:
    """Functional form of ProjectSubset."""
    return ProjectSubset.apply(x, geom, subset)
