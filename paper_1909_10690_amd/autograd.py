"""Differentiable MI for gradient-based registration (Eq. (3): T^ = argmax_T MI).

``MIFunction`` is a ``torch.autograd.Function`` over the physical fixed ->
moving 3x4 matrices P[n][12] of the candidate transforms.  Forward and
backward both run in the HIP library (``mi_grad``: Parzen forward table,
MI, dMI/dp tables, the backward sweep and the chain rule to the physical
entries); the backward here only contracts dL/dMI_q with dMI_q/dP.
:func:`centred_matrices` builds P from the centred parameters
p = (A.flat, t) of y = A (x - c) + c + t with torch operations, so autograd
carries the gradient on to them.
"""
from __future__ import annotations

import torch

from . import binding as B
from . import transforms as T


class MIFunction(torch.autograd.Function):
    """MI[n][n_q] of Parzen joint histograms as a function of P[n][12]."""

    @staticmethod
    def forward(ctx, P, gctx: B.Context, fixed: B.Volume, moving: B.Volume, bins: int, q, flags: int):
        mi, gP = gctx.grad(fixed, moving, P.detach().to(torch.float64), bins, q, flags=flags)
        ctx.save_for_backward(gP)
        return mi

    @staticmethod
    def backward(ctx, grad_mi):
        (gP,) = ctx.saved_tensors
        dP = (grad_mi.to(torch.float64).unsqueeze(-1) * gP).sum(dim=1)  # [n][12]
        return dP, None, None, None, None, None, None


def centred_matrices(params: torch.Tensor, centre) -> torch.Tensor:
    """P[n][12] = [A | c + t - A c] of centred parameters params[n][12] =
    (A.flat, t), differentiably."""
    A = params[:, :9].reshape(-1, 3, 3)
    t = params[:, 9:]
    c = torch.as_tensor(centre, dtype=params.dtype, device=params.device).reshape(3)
    off = c + t - (A @ c.unsqueeze(-1)).squeeze(-1)
    return torch.cat([A, off.unsqueeze(-1)], dim=2).reshape(-1, 12)


def identity_params(n: int = 1, device="cuda") -> torch.Tensor:
    p = torch.zeros((n, 12), dtype=torch.float64, device=device)
    p[:, [0, 4, 8]] = 1.0
    return p


def volume_centre(vol: B.Volume):
    """Physical centre of a volume (its spacing and origin applied)."""
    nz, ny, nx = vol.tensor.shape
    return T.fixed_centre((nx, ny, nz), vol.spacing, vol.origin)


def mutual_information(params: torch.Tensor, gctx: B.Context, fixed: B.Volume, moving: B.Volume,
                       bins: int, q=(1.0,), flags: int = B.BOUNDARY_CLAMP, centre=None) -> torch.Tensor:
    """Differentiable Parzen MI [n][len(q)] of centred parameters about
    ``centre`` (mm; the fixed volume's physical centre by default)."""
    c = volume_centre(fixed) if centre is None else centre
    return MIFunction.apply(centred_matrices(params, c), gctx, fixed, moving, bins, q, flags)
