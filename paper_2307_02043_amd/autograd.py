"""Differentiable mini-batch data term.

``ls_data(x, y, ctx, idx, scale)`` returns the scalar
F = scale * sum_b 1/2 ||H_b(x) - y_b||^2 (the mini-batch data term of
Section 4, eq. NewModelPro) as a torch tensor whose backward pass is the
library's adjoint Lippmann-Schwinger gradient.

With ``recompute=True`` (default) the forward pass runs only the forward
solves and keeps nothing but its inputs; backward calls the gradient, which
solves for the forward fields again before the adjoint solve, so memory
does not grow with the number of pending backward passes.  With
``recompute=False`` the forward pass computes the gradient right away and
stores it (one N^3 image) for backward.
"""
from __future__ import annotations

import torch


class LSData(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, y, lsctx, idx, scale, recompute):
        if recompute:
            loss, info = lsctx.loss(x, y, idx, scale)
            fctx.save_for_backward(x, y)
        else:
            g, loss, info = lsctx.grad(x, y, idx, scale)
            fctx.save_for_backward(g)
        fctx.lsctx, fctx.idx, fctx.scale, fctx.recompute = lsctx, idx, scale, recompute
        fctx.info = info
        return torch.tensor(loss, dtype=x.dtype, device=x.device)

    @staticmethod
    def backward(fctx, gout):
        if fctx.recompute:
            x, y = fctx.saved_tensors
            g, _, _ = fctx.lsctx.grad(x, y, fctx.idx, fctx.scale)
        else:
            (g,) = fctx.saved_tensors
        return g * gout, None, None, None, None, None


def ls_data(x: torch.Tensor, y: torch.Tensor, lsctx, idx, scale: float,
            recompute: bool = True) -> torch.Tensor:
    """Differentiable mini-batch data term (see the module docstring)."""
    return LSData.apply(x, y, lsctx, idx, scale, recompute)
