"""Differentiable MI for gradient-based registration (Eq. (3): T^ = argmax_T MI).

``MIFunction`` is a ``torch.autograd.Function`` over the 12 centred affine
parameters p = (A.flat, t) of each candidate transform,

    y_phys = A (x_phys - c) + c + t,

mapped to the library's index-space matrices by the constant Jacobian of
``transforms.index_jacobian``.  Forward and backward both run in the HIP
library (``mi_grad``: Parzen forward table, MI, dMI/dp table and the
backward sweep); the backward here only applies the chain rule
dL/dp = sum_q dL/dMI_q * J^T dMI_q/dM on 12-vectors.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from . import transforms as T


class Geometry:
    """Constant map from centred parameters to index-space matrices."""

    def __init__(self, fixed_shape_xyz, fixed_spacing=(1.0, 1.0, 1.0), fixed_origin=(0.0, 0.0, 0.0),
                 moving_spacing=(1.0, 1.0, 1.0), moving_origin=(0.0, 0.0, 0.0), device="cuda"):
        args = (fixed_shape_xyz, fixed_spacing, fixed_origin, moving_spacing, moving_origin)
        J = T.index_jacobian(*args)
        base = T.index_matrix(np.zeros((3, 3)), np.zeros(3), *args).reshape(12)
        self.J = torch.as_tensor(J, dtype=torch.float64, device=device)
        self.base = torch.as_tensor(base, dtype=torch.float64, device=device)

    def matrices(self, params: torch.Tensor) -> torch.Tensor:
        return params @ self.J.T + self.base

    def identity_params(self, n: int = 1) -> torch.Tensor:
        p = torch.zeros((n, 12), dtype=torch.float64, device=self.J.device)
        p[:, [0, 4, 8]] = 1.0
        return p


class MIFunction(torch.autograd.Function):
    """MI[n][n_q] of Parzen joint histograms as a function of params[n][12]."""

    @staticmethod
    def forward(ctx, params, gctx: B.Context, fixed: B.Volume, moving: B.Volume, geom: Geometry,
                bins: int, q, flags: int):
        M = geom.matrices(params.detach().to(torch.float64))
        mi, gM = gctx.grad(fixed, moving, M, bins, q, flags=flags)
        ctx.save_for_backward(gM)
        ctx.geom = geom
        return mi

    @staticmethod
    def backward(ctx, grad_mi):
        (gM,) = ctx.saved_tensors
        dM = (grad_mi.to(torch.float64).unsqueeze(-1) * gM).sum(dim=1)  # [n][12]
        return dM @ ctx.geom.J, None, None, None, None, None, None, None


def mutual_information(params: torch.Tensor, gctx: B.Context, fixed: B.Volume, moving: B.Volume,
                       geom: Geometry, bins: int, q=(1.0,), flags: int = B.BOUNDARY_CLAMP) -> torch.Tensor:
    """Differentiable Parzen MI, [n][len(q)]."""
    return MIFunction.apply(params, gctx, fixed, moving, geom, bins, q, flags)
