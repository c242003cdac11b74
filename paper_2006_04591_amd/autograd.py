"""The shearlet transform as a differentiable PyTorch layer.

The forward transform SH (shear_forward, Algorithm 1) is linear and real, so
the gradient of a loss with respect to its input is the adjoint applied to the
upstream gradient: dL/dx = SH^T dL/dc = SH* dL/dc (shear_adjoint, Algorithm 2
without the division by W). Both directions run the library's kernels on the
current stream; nothing here computes on the host.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from ._binding import ShearletSystem

__all__ = ["ShearletTransform", "ShearletLayer"]


class ShearletTransform(torch.autograd.Function):
    """c = SH x for x of shape (B, rows, cols); backward: grad_x = SH* grad_c."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, system: ShearletSystem) -> torch.Tensor:
        ctx.system = system
        return system.forward(x.contiguous())

    @staticmethod
    def backward(ctx, grad_c: torch.Tensor):
        grad_x = ctx.system.adjoint(grad_c.contiguous()) if ctx.needs_input_grad[0] else None
        return grad_x, None


class ShearletLayer(torch.nn.Module):
    """Fixed (non-trainable) shearlet decomposition layer: (B, 1, rows, cols) or (B, rows, cols) float32
    -> (B, K, rows, cols), differentiable with respect to its input."""

    def __init__(self, rows: int, cols: int, n_scales: int, shear_levels: Optional[Sequence[int]] = None,
                 system: Optional[ShearletSystem] = None):
        super().__init__()
        self.system = system if system is not None else ShearletSystem.build(rows, cols, n_scales, shear_levels)
        if (self.system.rows, self.system.cols) != (rows, cols):
            raise ValueError("system size does not match the layer size")

    @property
    def K(self) -> int:
        return self.system.K

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        if x.dim() == 4:
            if x.shape[1] != 1:
                raise ValueError(f"expected one input channel, got {x.shape[1]}")
            x = x[:, 0]
        if x.dim() != 3:
            raise ValueError(f"expected (B, rows, cols) or (B, 1, rows, cols), got {tuple(x.shape)}")
        return ShearletTransform.apply(x, self.system)
