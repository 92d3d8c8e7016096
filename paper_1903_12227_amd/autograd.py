"""torch.autograd wrappers of the homogenized matrix.

The energy form of A_hom is stationary in the correctors (each corrector
solves its Galerkin system, eqn. wg03), so its derivative with respect to a
cell value is the cell integral of (e_i + grad phi_i).(e_j + grad phi_j) / n^2
at the converged correctors: the backward pass is one librve kernel, with no
adjoint solve.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api


class RveAhom(torch.autograd.Function):
    """A_hom (B, 2, 2) as a differentiable function of the per-cell field a."""

    @staticmethod
    def forward(ctx, a: torch.Tensor, h: float, opts: Optional[api.Options]):
        res = api.solve_batch(a.detach().contiguous(), h, opts, want_phi=True, want_flux=False)
        ctx.save_for_backward(a, res.phi)
        ctx.h = h
        ctx.scheme = opts.scheme if opts is not None else 0
        return res.ahom

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        a, phi = ctx.saved_tensors
        g, _ = api.grad(a.detach().contiguous(), phi, ctx.h, G.contiguous(), scheme=ctx.scheme)
        return g, None, None


class RveAhomContrast(torch.autograd.Function):
    """A_hom as a function of the inclusion value `contrast` (a 0-d or (B,)
    tensor): the caller's field `a` holds that value on the inclusion cells,
    and d A / d contrast sums the per-cell derivative over those cells."""

    @staticmethod
    def forward(ctx, contrast: torch.Tensor, a: torch.Tensor, h: float, opts: Optional[api.Options]):
        res = api.solve_batch(a.detach().contiguous(), h, opts, want_phi=True, want_flux=False)
        ctx.save_for_backward(a, res.phi, contrast)
        ctx.h = h
        ctx.scheme = opts.scheme if opts is not None else 0
        return res.ahom

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        a, phi, contrast = ctx.saved_tensors
        vals = contrast.detach().reshape(-1).cpu()
        if vals.numel() != 1 and not bool(torch.all(vals == vals[0])):
            raise ValueError("RveAhomContrast needs one contrast value for the batch")
        _, gin = api.grad(a.detach().contiguous(), phi, ctx.h, G.contiguous(), a_in=float(vals[0]),
                          scheme=ctx.scheme)
        if contrast.dim() == 0:
            return gin.sum().reshape(()), None, None, None
        return gin.reshape(contrast.shape), None, None, None


def ahom(a: torch.Tensor, h: float = 1.0, opts: Optional[api.Options] = None) -> torch.Tensor:
    return RveAhom.apply(a, h, opts)
