"""Gradient-based registration driver (Eq. (3): T^ = argmax_T F_m(u, v o T)).

The Optimizer block of Fig. 1 as a thin loop around ``mi_grad``: each step
is one Parzen forward + backward on the device and an Adam ascent step on
the 12 centred affine parameters (A, t).  ``mixed=True`` follows the
strategy proposed in the Discussion: one histogram yields both entropies,
so translation parameters follow the Tsallis-MI gradient and the linear
part (rotation, scale, skew) the Shannon-MI gradient.

The optimiser state (parameters, step, Adam moments) can be written to and
resumed from a JSON checkpoint.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .autograd import Geometry


@dataclass
class RegState:
    params: list          # 12 floats: A (row-major 3x3), t (3)
    step: int = 0
    m: list = field(default_factory=lambda: [0.0] * 12)
    v: list = field(default_factory=lambda: [0.0] * 12)
    history: list = field(default_factory=list)  # (step, MI per entropy)

    def save(self, path: str) -> None:
        with open(path, "w") as f:
            json.dump(self.__dict__, f)

    @classmethod
    def load(cls, path: str) -> "RegState":
        with open(path) as f:
            return cls(**json.load(f))


def register(gctx: B.Context, fixed: B.Volume, moving: B.Volume, geom: Geometry, bins: int,
             params0, steps: int = 200, q_translation: float = 1.3, mixed: bool = True,
             lr_linear: float = 2e-3, lr_translation: float = 0.2, betas=(0.9, 0.999),
             flags: int = B.BOUNDARY_CLAMP, state: RegState | None = None,
             checkpoint: str | None = None, every: int = 50, workspace=None) -> RegState:
    """Maximises Parzen MI over the centred affine parameters.

    With ``mixed`` the objective's gradient takes the linear entries from
    Shannon MI and the translation entries from Tsallis MI at
    ``q_translation``; otherwise every entry follows Tsallis MI at that q.
    """
    dev = fixed.tensor.device
    if state is None:
        state = RegState(params=[float(x) for x in np.asarray(params0, dtype=np.float64).reshape(12)])
    q = [1.0, q_translation]
    lr = np.array([lr_linear] * 9 + [lr_translation] * 3)
    b1, b2 = betas
    p = torch.tensor(state.params, dtype=torch.float64, device=dev).reshape(1, 12)
    if workspace is None:
        workspace = gctx.workspace(gctx.workspace_size(fixed, moving, 1, bins, len(q), flags | B.HIST_PARZEN, True))
    m = np.asarray(state.m, dtype=np.float64)
    v = np.asarray(state.v, dtype=np.float64)
    J = geom.J
    while state.step < steps:
        M = geom.matrices(p)
        mi, gM = gctx.grad(fixed, moving, M, bins, q, flags=flags, workspace=workspace)
        gp = (gM[0] @ J).cpu().numpy()          # [n_q][12] d MI_q / d params
        if mixed:
            g = np.concatenate([gp[0, :9], gp[1, 9:]])
        else:
            g = gp[1]
        state.step += 1
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** state.step)
        vh = v / (1 - b2 ** state.step)
        delta = lr * mh / (np.sqrt(vh) + 1e-12)
        p += torch.as_tensor(delta, dtype=torch.float64, device=dev).reshape(1, 12)   # ascent
        state.params = [float(x) for x in p.reshape(12).cpu().numpy()]
        state.m, state.v = [float(x) for x in m], [float(x) for x in v]
        state.history.append((state.step, [float(x) for x in mi[0].cpu().numpy()]))
        if checkpoint and (state.step % every == 0 or state.step == steps):
            state.save(checkpoint)
        if not all(math.isfinite(x) for x in state.params):
            raise FloatingPointError("registration diverged")
    return state
