"""torch.autograd wrappers of the homogenized matrix.

The energy form of A_hom is stationary in the correctors (each corrector
solves its Galerkin system, eqn. wg03), so its derivative with respect to a
cell value is the cell integral of (e_i + grad phi_i).(e_j + grad phi_j) / n^2
at the converged correctors: the backward pass is one librve kernel, with no
adjoint solve. A forward solve that does not converge, or that meets an
invalid coefficient, raises: the stationarity identity holds only at the
converged correctors.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _native as N
from . import api


def _solved(a: torch.Tensor, h: float, opts: Optional[api.Options]) -> api.Result:
    res = api.solve_batch(a, h, opts, want_phi=True, want_flux=False)
    if res.code != N.OK:
        bad = torch.nonzero(res.status != N.OK).flatten().tolist()
        raise N.RveError(res.code, f"A_hom forward solve (items {bad})")
    return res


class RveAhom(torch.autograd.Function):
    """A_hom (B, 2, 2) as a differentiable function of the per-cell field a
    (B, n, n); a single field (n, n) gives (2, 2)."""

    @staticmethod
    def forward(ctx, a: torch.Tensor, h: float, opts: Optional[api.Options]):
        single = a.dim() == 2
        a3 = (a.unsqueeze(0) if single else a).detach().contiguous()
        res = _solved(a3, h, opts)
        ctx.save_for_backward(a3, res.phi)
        ctx.h = h
        ctx.single = single
        ctx.scheme = opts.scheme if opts is not None else 0
        return res.ahom[0] if single else res.ahom

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        a3, phi = ctx.saved_tensors
        G3 = (G.unsqueeze(0) if ctx.single else G).contiguous()
        g, _, _ = api.grad(a3, phi, ctx.h, G3, scheme=ctx.scheme)
        return (g[0] if ctx.single else g), None, None


class RveAhomContrast(torch.autograd.Function):
    """A_hom (B, 2, 2) of the two-valued fields a = contrast on the covered
    cells (mask (B, n, n), bool or uint8) and a_bg elsewhere (Sec. 2, eqns.
    Stoch-decomp and ahm_coef), as a function of `contrast`: a 0-d tensor
    (one value for the batch) or a (B,) tensor (one per realization). The
    fields are built on the device from the mask, so the forward solve and
    the derivative (the per-cell derivative summed over the covered cells)
    use the same covered set."""

    @staticmethod
    def forward(ctx, contrast: torch.Tensor, mask: torch.Tensor, a_bg: float, h: float,
                opts: Optional[api.Options]):
        B = mask.shape[0]
        if contrast.dim() not in (0, 1) or (contrast.dim() == 1 and contrast.shape != (B,)):
            raise ValueError("contrast must be a 0-d tensor or have shape (B,)")
        values = contrast.detach().to(device=mask.device, dtype=torch.float64).expand(B).contiguous()
        a = api.field_from_mask(mask, values, a_bg)
        res = _solved(a, h, opts)
        ctx.save_for_backward(a, res.phi, mask.contiguous())
        ctx.h = h
        ctx.scalar = contrast.dim() == 0
        ctx.scheme = opts.scheme if opts is not None else 0
        return res.ahom

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        a, phi, mask = ctx.saved_tensors
        _, gin, gsum = api.grad(a, phi, ctx.h, G.contiguous(), mask=mask, want_sum=ctx.scalar, scheme=ctx.scheme)
        return (gsum.reshape(()) if ctx.scalar else gin), None, None, None, None


def ahom(a: torch.Tensor, h: float = 1.0, opts: Optional[api.Options] = None) -> torch.Tensor:
    return RveAhom.apply(a, h, opts)


def ahom_contrast(contrast: torch.Tensor, mask: torch.Tensor, a_bg: float = 1.0, h: float = 1.0,
                  opts: Optional[api.Options] = None) -> torch.Tensor:
    return RveAhomContrast.apply(contrast, mask, a_bg, h, opts)
