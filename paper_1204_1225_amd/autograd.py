"""Differentiable Kirchhoff operators.

KirchhoffDemigrate: forward = demigration L (image -> traces, Kirchhoff
modelling), backward = migration L^T (the transpose of Eq. (1)'s
discretisation), so gradients of data-space losses flow to the image.
KirchhoffMigrate is the mirror pair.  Both kernels evaluate every
(trace, image point) pair identically, so each backward is the exact
adjoint of its forward up to float32 summation rounding.
"""
from __future__ import annotations

import torch

from . import ops


class KirchhoffDemigrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, dp: "ops.DeviceProblem"):
        ctx.dp = dp
        return ops.demigrate(dp, image.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        g = ops.migrate(ctx.dp, data=grad_traces.detach().contiguous().to(torch.float32), dtype="f32")
        return g, None


class KirchhoffMigrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, traces: torch.Tensor, dp: "ops.DeviceProblem"):
        ctx.dp = dp
        return ops.migrate(dp, data=traces.detach().contiguous().to(torch.float32), dtype="f32")

    @staticmethod
    def backward(ctx, grad_image: torch.Tensor):
        return ops.demigrate(ctx.dp, grad_image.detach().contiguous()), None


def demigrate(image: torch.Tensor, dp: "ops.DeviceProblem") -> torch.Tensor:
    return KirchhoffDemigrate.apply(image, dp)


def migrate(traces: torch.Tensor, dp: "ops.DeviceProblem") -> torch.Tensor:
    return KirchhoffMigrate.apply(traces, dp)
