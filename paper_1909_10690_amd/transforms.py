"""Affine transform parameterisations -> physical 3x4 matrices.

The library takes, per candidate transform, a 3x4 matrix ``P`` that maps a
point of the fixed volume (mm) to a point of the moving volume (mm): the
Transform block of Fig. 1, ``v(T(x))``; each volume carries its own voxel
spacing and origin, and the library composes the voxel-index map itself.
This module builds ``P`` from the centred parameterisation used in
registration (Introduction: translation, rotation, scale and skew form the
affine family; 12 degrees of freedom, Methodology):

    y = A (x - c) + c + t,   i.e.   P = [A | c + t - A c],

with ``c`` a physical centre, by default that of the fixed volume.  ``P``
is affine in the 12 centred parameters (the 9 entries of A and the 3 of
t), so gradients with respect to ``P`` map to gradients with respect to
(A, t) through a constant Jacobian (:func:`centred_jacobian`).

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
    """Physical centre of a volume: origin + (n - 1) / 2 * spacing."""
    n = np.asarray(shape_xyz, dtype=np.float64)
    return np.asarray(origin, dtype=np.float64) + (n - 1.0) / 2.0 * np.asarray(spacing, dtype=np.float64)


def centred_matrix(A, t, centre) -> np.ndarray:
    """Physical 3x4 matrix of y = A (x - c) + c + t."""
    A = np.asarray(A, dtype=np.float64).reshape(3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    c = np.asarray(centre, dtype=np.float64).reshape(3)
    P = np.zeros((3, 4))
    P[:, :3] = A
    P[:, 3] = c + t - A @ c
    return P


def centred_matrices(A, t, centre) -> np.ndarray:
    """:func:`centred_matrix` of a batch: A [n][3][3], t [n][3] -> [n][12]."""
    A = np.asarray(A, dtype=np.float64).reshape(-1, 3, 3)
    t = np.asarray(t, dtype=np.float64).reshape(-1, 3)
    c = np.asarray(centre, dtype=np.float64).reshape(3)
    P = np.zeros((A.shape[0], 3, 4))
    P[:, :, :3] = A
    P[:, :, 3] = c + t - A @ c
    return P.reshape(-1, 12)


def centred_jacobian(centre) -> np.ndarray:
    """J[e, p] = d P.flat[e] / d params[p], params = (A.flat (9), t (3)).

    P is affine in the parameters, so J is constant: d P[r][c] / d A[r][c] = 1,
    d P[r][3] / d A[r][c] = -centre[c], d P[r][3] / d t[r] = 1."""
    c = np.asarray(centre, dtype=np.float64).reshape(3)
    J = np.zeros((12, 12))
    for r in range(3):
        for k in range(3):
            J[4 * r + k, 3 * r + k] = 1.0
            J[4 * r + 3, 3 * r + k] = -c[k]
        J[4 * r + 3, 9 + r] = 1.0
    return J


def params_from(A, t) -> np.ndarray:
    return np.concatenate([np.asarray(A, dtype=np.float64).reshape(9), np.asarray(t, dtype=np.float64).reshape(3)])


def translation(t) -> np.ndarray:
    """Pure translation y = x + t."""
    M = np.zeros((3, 4))
    M[:, :3] = np.eye(3)
    M[:, 3] = np.asarray(t, dtype=np.float64)
    return M
