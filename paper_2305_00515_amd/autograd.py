"""torch.autograd.Function over the fp32 HIP kernels (edge-magnitude loss).

Forward calls sobel4x5_f32_fwd, backward calls the hand-written adjoint
sobel4x5_f32_bwd; only the input image is saved (the responses are
recomputed in the backward kernel).
"""
from __future__ import annotations

import torch

from . import api


class Sobel4x5Magnitude(torch.autograd.Function):
    """M = sqrt(Gx^2 + Gd^2 + Gy^2 + Gdt^2) of an fp32 image batch (B, H, W) or (H, W)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, border: int = api.BORDER_REPLICATE):
        if x.dtype != torch.float32 or not x.is_cuda:
            raise TypeError("Sobel4x5Magnitude needs a float32 GPU tensor")
        x = x.contiguous()
        ctx.border = border
        ctx.save_for_backward(x)
        return api.sobel4x5_f32_fwd(x, border)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (x,) = ctx.saved_tensors
        g = grad_out.contiguous()
        if g.dtype != torch.float32:
            g = g.float()
        return api.sobel4x5_f32_bwd(x, g, ctx.border), None


def sobel4x5_magnitude(x: torch.Tensor, border: int = api.BORDER_REPLICATE) -> torch.Tensor:
    return Sobel4x5Magnitude.apply(x, border)
