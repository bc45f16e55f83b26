"""Affine transform parameterisations -> index-space 3x4 matrices.

The library takes, per candidate transform, a 3x4 matrix ``M`` that maps a
fixed-volume voxel index (i, j, k) to a continuous moving-volume voxel index
(the Transform block of Fig. 1: ``v(T(x))``).  This module builds those
matrices from the physical, centred parameterisation used in registration
(Introduction: translation, rotation, scale and skew form the affine family;
12 degrees of freedom, Methodology):

    y_phys = A (x_phys - c) + c + t,   x_phys = o_f + S_f i,   y_idx = S_m^-1 (y_phys - o_m)

with ``c`` the physical centre of the fixed volume.  ``M`` is linear in the
12 centred parameters (the 9 entries of A and the 3 of t), so gradients with
respect to ``M`` map to gradients with respect to (A, t) through a constant
Jacobian (:func:`index_jacobian`).

The matrices are host-side inputs shared by the GPU library and the CPU
oracle as data; nothing here computes any part of the metric.
"""
from __future__ import annotations

import numpy as np


def rotation_matrix(angles_deg) -> np.ndarray:
    """R = Rz @ Ry @ Rx for Euler angles (degrees) about x, y, z."""
    ax, ay, az = np.deg2rad(np.asarray(angles_deg, dtype=np.float64))
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def affine_matrix(angles_deg=(0.0, 0.0, 0.0), scale=(1.0, 1.0, 1.0), shear=(0.0, 0.0, 0.0)) -> np.ndarray:
    """A = R(angles) @ Shear(h_xy, h_xz, h_yz) @ diag(scale)."""
    s = np.broadcast_to(np.asarray(scale, dtype=np.float64), (3,))
    hxy, hxz, hyz = shear
    H = np.array([[1.0, hxy, hxz], [0.0, 1.0, hyz], [0.0, 0.0, 1.0]])
    return rotation_matrix(angles_deg) @ H @ np.diag(s)


def fixed_centre(shape_xyz, spacing=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    n = np.asarray(shape_xyz, dtype=np.float64)
    return np.asarray(origin, dtype=np.float64) + (n - 1.0) / 2.0 * np.asarray(spacing, dtype=np.float64)


def index_matrix(A, t, fixed_shape_xyz, fixed_spacing=(1.0, 1.0, 1.0), fixed_origin=(0.0, 0.0, 0.0),
                 moving_spacing=(1.0, 1.0, 1.0), moving_origin=(0.0, 0.0, 0.0), centre=None) -> np.ndarray:
    """Index-space 3x4 matrix (fixed voxel index -> moving voxel index)."""
    A = np.asarray(A, dtype=np.float64).reshape(3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    Sf = np.diag(np.asarray(fixed_spacing, dtype=np.float64))
    Sm_inv = np.diag(1.0 / np.asarray(moving_spacing, dtype=np.float64))
    of = np.asarray(fixed_origin, dtype=np.float64)
    om = np.asarray(moving_origin, dtype=np.float64)
    c = fixed_centre(fixed_shape_xyz, fixed_spacing, fixed_origin) if centre is None else np.asarray(centre, dtype=np.float64)
    lin = Sm_inv @ A @ Sf
    off = Sm_inv @ (A @ (of - c) + c + t - om)
    M = np.zeros((3, 4))
    M[:, :3] = lin
    M[:, 3] = off
    return M


def index_matrices(A, t, fixed_shape_xyz, fixed_spacing=(1.0, 1.0, 1.0), fixed_origin=(0.0, 0.0, 0.0),
                   moving_spacing=(1.0, 1.0, 1.0), moving_origin=(0.0, 0.0, 0.0), centre=None) -> np.ndarray:
    """:func:`index_matrix` of a batch: A [n][3][3], t [n][3] -> [n][12]."""
    A = np.asarray(A, dtype=np.float64).reshape(-1, 3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(-1, 3)
    Sf = np.diag(np.asarray(fixed_spacing, dtype=np.float64))
    Sm_inv = np.diag(1.0 / np.asarray(moving_spacing, dtype=np.float64))
    of = np.asarray(fixed_origin, dtype=np.float64)
    om = np.asarray(moving_origin, dtype=np.float64)
    c = fixed_centre(fixed_shape_xyz, fixed_spacing, fixed_origin) if centre is None else np.asarray(centre, dtype=np.float64)
    M = np.zeros((A.shape[0], 3, 4))
    M[:, :, :3] = Sm_inv @ A @ Sf
    M[:, :, 3] = ((A @ (of - c)) + c + t - om) @ Sm_inv.T
    return M.reshape(-1, 12)


def index_jacobian(fixed_shape_xyz, fixed_spacing=(1.0, 1.0, 1.0), fixed_origin=(0.0, 0.0, 0.0),
                   moving_spacing=(1.0, 1.0, 1.0), moving_origin=(0.0, 0.0, 0.0), centre=None) -> np.ndarray:
    """J[e, p] = d M.flat[e] / d params[p], params = (A.flat (9), t (3)).

    M depends linearly (affinely) on the parameters, so J is constant."""
    J = np.zeros((12, 12))
    base = index_matrix(np.zeros((3, 3)), np.zeros(3), fixed_shape_xyz, fixed_spacing, fixed_origin,
                        moving_spacing, moving_origin, centre).reshape(12)
    for p in range(12):
        e = np.zeros(12)
        e[p] = 1.0
        M = index_matrix(e[:9].reshape(3, 3), e[9:], fixed_shape_xyz, fixed_spacing, fixed_origin,
                         moving_spacing, moving_origin, centre).reshape(12)
        J[:, p] = M - base
    return J


def params_from(A, t) -> np.ndarray:
    return np.concatenate([np.asarray(A, dtype=np.float64).reshape(9), np.asarray(t, dtype=np.float64).reshape(3)])


def translation(t) -> np.ndarray:
    """Pure index-space translation y = x + t."""
    M = np.zeros((3, 4))
    M[:, :3] = np.eye(3)
    M[:, 3] = np.asarray(t, dtype=np.float64)
    return M
