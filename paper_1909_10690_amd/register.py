"""Gradient-based registration driver (Eq. (3): T^ = argmax_T F_m(u, v o T)).

The Optimizer block of Fig. 1 as a thin loop around ``mi_grad``: each step
is one Parzen forward + backward on the device and an Adam ascent step on
the 12 centred affine parameters (A, t).  ``mixed=True`` follows the
strategy proposed in the Discussion: one histogram yields both entropies,
so translation parameters follow the Tsallis-MI gradient and the linear
part (rotation, scale, skew) the Shannon-MI gradient.

Two parameterisations of the linear part: ``"affine"`` steps the 9 entries
of A directly; ``"decomposed"`` steps A = R(angles) H(shears) diag(exp(s))
(the factorisation of ``transforms.affine_matrix``), so that a rotation is a
coordinate of its own.  Adam normalises each coordinate separately, and on
anatomy whose rotations a shear can nearly undo, the MI ridge runs along
the antisymmetric combination of two raw entries, where per-entry steps
make little progress.

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
from . import transforms as T
from .autograd import volume_centre


def decomposed_to_affine(d) -> np.ndarray:
    """(angles (rad), log-scales, shears (h_xy, h_xz, h_yz), t) -> (A.flat, t),
    A = Rz Ry Rx H S as in ``transforms.affine_matrix``, written out in
    scalars (the registration computes it before every sweep)."""
    ax, ay, az, l0, l1, l2, hxy, hxz, hyz, t0, t1, t2 = (float(x) for x in np.asarray(d, dtype=np.float64))
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    # R = Rz Ry Rx
    r00, r01, r02 = cz * cy, cz * sy * sx - sz * cx, cz * sy * cx + sz * sx
    r10, r11, r12 = sz * cy, sz * sy * sx + cz * cx, sz * sy * cx - cz * sx
    r20, r21, r22 = -sy, cy * sx, cy * cx
    # columns of R H, then scaled by S
    s0, s1, s2 = math.exp(l0), math.exp(l1), math.exp(l2)
    return np.array([
        r00 * s0, (r00 * hxy + r01) * s1, (r00 * hxz + r01 * hyz + r02) * s2,
        r10 * s0, (r10 * hxy + r11) * s1, (r10 * hxz + r11 * hyz + r12) * s2,
        r20 * s0, (r20 * hxy + r21) * s1, (r20 * hxz + r21 * hyz + r22) * s2,
        t0, t1, t2])


def affine_to_decomposed(p) -> np.ndarray:
    """Inverse of decomposed_to_affine for det(A) > 0: A = Q U by QR with
    U's diagonal made positive, Q = Rz Ry Rx, U = H diag(s)."""
    p = np.asarray(p, dtype=np.float64)
    A = p[:9].reshape(3, 3)
    if not np.linalg.det(A) > 0:
        raise ValueError("the linear part must have a positive determinant")
    Q, U = np.linalg.qr(A)
    sg = np.sign(np.diag(U))
    Q, U = Q * sg, sg[:, None] * U
    s = np.diag(U)
    hxy, hxz, hyz = U[0, 1] / s[1], U[0, 2] / s[2], U[1, 2] / s[2]
    ay = -np.arcsin(np.clip(Q[2, 0], -1.0, 1.0))
    ax = np.arctan2(Q[2, 1], Q[2, 2])
    az = np.arctan2(Q[1, 0], Q[0, 0])
    return np.concatenate([[ax, ay, az], np.log(s), [hxy, hxz, hyz], p[9:12]])


def decomposed_jacobian(d) -> np.ndarray:
    """J[i, j] = d affine_params[i] / d d[j], analytically: with
    A = Rz Ry Rx H S (S = diag(exp(log-scales)), H the unit upper-triangular
    shear), an angle differentiates its own rotation factor, log-scale i
    scales column i of A, and a shear entry moves one entry of H; t maps to
    itself.  (Central differences took ~0.6 ms of host time a call, most of
    a registration iteration's host share.)"""
    d = np.asarray(d, dtype=np.float64)
    ax, ay, az = d[0:3]
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    dRx = np.array([[0, 0, 0], [0, -sx, -cx], [0, cx, -sx]])
    dRy = np.array([[-sy, 0, cy], [0, 0, 0], [-cy, 0, -sy]])
    dRz = np.array([[-sz, -cz, 0], [cz, -sz, 0], [0, 0, 0]])
    hxy, hxz, hyz = d[6:9]
    H = np.array([[1.0, hxy, hxz], [0.0, 1.0, hyz], [0.0, 0.0, 1.0]])
    S = np.diag(np.exp(d[3:6]))
    R = Rz @ Ry @ Rx
    J = np.zeros((12, 12))
    J[:9, 0] = (Rz @ Ry @ dRx @ H @ S).reshape(9)
    J[:9, 1] = (Rz @ dRy @ Rx @ H @ S).reshape(9)
    J[:9, 2] = (dRz @ Ry @ Rx @ H @ S).reshape(9)
    A = R @ H @ S
    for i in range(3):
        dA = np.zeros((3, 3))
        dA[:, i] = A[:, i]
        J[:9, 3 + i] = dA.reshape(9)
    for j, (r, c) in enumerate(((0, 1), (0, 2), (1, 2))):
        E = np.zeros((3, 3))
        E[r, c] = 1.0
        J[:9, 6 + j] = (R @ E @ S).reshape(9)
    J[9:, 9:] = np.eye(3)
    return J


@dataclass
class RegState:
    params: list          # 12 floats in the parameterisation `param`
    step: int = 0
    param: str = "affine"  # "affine": A (row-major 3x3), t; "decomposed": see decomposed_to_affine
    m: list = field(default_factory=lambda: [0.0] * 12)
    v: list = field(default_factory=lambda: [0.0] * 12)
    history: list = field(default_factory=list)  # (step, MI per entropy)

    def affine(self) -> np.ndarray:
        """The state's transform as 12 centred affine parameters (A.flat, t)."""
        p = np.asarray(self.params, dtype=np.float64)
        return decomposed_to_affine(p) if self.param == "decomposed" else p

    def save(self, path: str) -> None:
        with open(path, "w") as f:
            json.dump(self.__dict__, f)

    @classmethod
    def load(cls, path: str) -> "RegState":
        with open(path) as f:
            return cls(**json.load(f))


def register(gctx: B.Context, fixed: B.Volume, moving: B.Volume, bins: int,
             params0, steps: int = 200, q_translation: float = 1.3, mixed: bool = True,
             lr_linear: float = 2e-3, lr_translation: float = 0.2, betas=(0.9, 0.999),
             flags: int = B.BOUNDARY_CLAMP, state: RegState | None = None,
             checkpoint: str | None = None, every: int = 50, workspace=None,
             param: str = "affine", centre=None) -> RegState:
    """Maximises Parzen MI over the centred affine parameters ``params0``
    (A.flat, t) of y = A (x - c) + c + t, c = ``centre`` (mm; the fixed
    volume's physical centre by default), stepping them in the
    parameterisation ``param``.

    With ``mixed`` the objective's gradient takes the linear entries from
    Shannon MI and the translation entries from Tsallis MI at
    ``q_translation``; otherwise every entry follows Tsallis MI at that q.
    A resumed ``state`` keeps its own parameterisation.
    """
    dev = fixed.tensor.device
    if state is None:
        if param not in ("affine", "decomposed"):
            raise ValueError(f"unknown parameterisation {param!r}")
        p0 = np.asarray(params0, dtype=np.float64).reshape(12)
        if param == "decomposed":
            p0 = affine_to_decomposed(p0)
        state = RegState(params=[float(x) for x in p0], param=param)
    dec = state.param == "decomposed"
    q = [1.0, q_translation]
    lr = np.array([lr_linear] * 9 + [lr_translation] * 3)
    b1, b2 = betas
    d = np.asarray(state.params, dtype=np.float64)
    if workspace is None:
        workspace = gctx.workspace(gctx.workspace_size(fixed, moving, 1, bins, len(q), flags | B.HIST_PARZEN | B.GRADIENT))
    m = np.asarray(state.m, dtype=np.float64)
    v = np.asarray(state.v, dtype=np.float64)
    c = volume_centre(fixed) if centre is None else np.asarray(centre, dtype=np.float64)
    J = T.centred_jacobian(c)              # d P / d (A, t), constant
    first = state.step
    nq = len(q)
    # per step one host -> device copy of P (from pinned memory) and one
    # device -> host copy of MI and dMI/dP together (one buffer)
    P_host = torch.empty((1, 12), dtype=torch.float64, pin_memory=dev.type == "cuda")
    P_dev = torch.empty((1, 12), dtype=torch.float64, device=dev)
    res = torch.empty(nq * 13, dtype=torch.float64, device=dev)
    mi_out, g_out = res[:nq].view(1, nq), res[nq:].view(1, nq, 12)
    grad = gctx.grad_fn(fixed, moving, P_dev, bins, q, flags, workspace, (mi_out, g_out))

    def sync_state():
        state.params = [float(x) for x in d]
        state.m, state.v = [float(x) for x in m], [float(x) for x in v]

    while state.step < steps:
        pa = decomposed_to_affine(d) if dec else d
        P_host.numpy()[:] = T.centred_matrix(pa[:9], pa[9:], c).reshape(1, 12)
        P_dev.copy_(P_host, non_blocking=True)
        # the volumes and workspace stay the same over the loop: after the
        # first call the library reuses their preparation
        grad(B.VOLUMES_UNCHANGED if state.step > first else 0)
        # while the device sweeps: the chain rule's Jacobian at this step
        Jd = J @ decomposed_jacobian(d) if dec else J   # d P / d (angles, log-scales, shears, t) or d (A, t)
        h = res.cpu().numpy()                   # waits for the step; P_host is free again
        mi, gP = h[:nq], h[nq:].reshape(nq, 12)
        gp = gP @ Jd                            # [n_q][12] d MI_q / d parameters
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
        d = d + delta   # ascent
        state.history.append((state.step, [float(x) for x in mi]))
        if checkpoint and (state.step % every == 0 or state.step == steps):
            sync_state()
            state.save(checkpoint)
        if not np.all(np.isfinite(d)):
            sync_state()
            raise FloatingPointError("registration diverged")
    sync_state()
    return state
