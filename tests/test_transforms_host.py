"""Host-side transform construction (Introduction / Methodology: the affine
family of 12 degrees of freedom, applied about the fixed volume's centre;
Fig. 1: the Transform block maps fixed voxels into the moving volume),
checked on the CPU against the physical definition point by point and
against closed forms.

* The index-space matrix sends fixed voxel i to the moving index of the
  same physical point: x = o_f + s_f i, y = A (x - c) + c + t,
  m = (y - o_m) / s_m; the batch builder agrees with the single one, and
  ``Geometry.matrices`` (the autograd path's linear map) with both.
* Euler rotations are proper rotations; with no rotation and no shear the
  affine matrix is diag(scale).
* The registration parameterisation (angles, log-scales, shears, t) round
  trips, and its Jacobian at the identity has the closed-form columns: the
  rotation generators, the unit diagonal entries, the unit translations.
"""
import numpy as np
import pytest

from paper_1909_10690_amd import transforms as T


def geometry(rng):
    shape = tuple(int(v) for v in rng.integers(2, 40, 3))
    return dict(fixed_shape_xyz=shape, fixed_spacing=rng.uniform(0.5, 2.0, 3), fixed_origin=rng.uniform(-50, 50, 3),
                moving_spacing=rng.uniform(0.5, 2.0, 3), moving_origin=rng.uniform(-50, 50, 3))


def test_index_matrix_follows_physical_points():
    rng = np.random.default_rng(11)
    for _ in range(20):
        g = geometry(rng)
        A = T.affine_matrix(rng.uniform(-30, 30, 3), rng.uniform(0.8, 1.2, 3), rng.uniform(-0.1, 0.1, 3))
        t = rng.uniform(-10, 10, 3)
        M = T.index_matrix(A, t, **g)
        n = np.asarray(g["fixed_shape_xyz"], dtype=np.float64)
        c = g["fixed_origin"] + (n - 1) / 2 * g["fixed_spacing"]
        for _ in range(10):
            i = rng.integers(0, n).astype(np.float64)
            x = g["fixed_origin"] + g["fixed_spacing"] * i
            y = A @ (x - c) + c + t
            m = (y - g["moving_origin"]) / g["moving_spacing"]
            assert np.allclose(M[:, :3] @ i + M[:, 3], m, rtol=0, atol=1e-9)


def test_batch_and_autograd_builders_agree():
    import torch
    from paper_1909_10690_amd.autograd import Geometry
    rng = np.random.default_rng(12)
    g = geometry(rng)
    A = np.stack([T.affine_matrix(rng.uniform(-20, 20, 3), rng.uniform(0.9, 1.1, 3)) for _ in range(6)])
    t = rng.uniform(-5, 5, (6, 3))
    Mb = T.index_matrices(A, t, **g)
    for k in range(6):
        assert np.allclose(Mb[k], T.index_matrix(A[k], t[k], **g).reshape(12), rtol=0, atol=1e-12)
    geo = Geometry(g["fixed_shape_xyz"], g["fixed_spacing"], g["fixed_origin"], g["moving_spacing"],
                   g["moving_origin"], "cpu")
    P = torch.as_tensor(np.concatenate([A.reshape(6, 9), t], axis=1))
    assert np.allclose(geo.matrices(P).numpy(), Mb, rtol=0, atol=1e-9)


def test_rotations_and_plain_scale():
    rng = np.random.default_rng(13)
    for _ in range(50):
        R = T.rotation_matrix(rng.uniform(-180, 180, 3))
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and abs(np.linalg.det(R) - 1) < 1e-12
    s = np.array([0.9, 1.3, 2.0])
    assert np.allclose(T.affine_matrix((0, 0, 0), s, (0, 0, 0)), np.diag(s), atol=0)
    # a rotation about z by 90 degrees sends x to y
    assert np.allclose(T.rotation_matrix((0, 0, 90)) @ [1, 0, 0], [0, 1, 0], atol=1e-15)


def test_decomposed_parameters_round_trip():
    from paper_1909_10690_amd.register import affine_to_decomposed, decomposed_to_affine
    rng = np.random.default_rng(14)
    for _ in range(100):
        d = np.concatenate([rng.uniform(-0.6, 0.6, 3), rng.uniform(-0.2, 0.2, 3), rng.uniform(-0.2, 0.2, 3),
                            rng.uniform(-10, 10, 3)])
        assert np.allclose(affine_to_decomposed(decomposed_to_affine(d)), d, rtol=0, atol=1e-10)
    with pytest.raises(ValueError):
        affine_to_decomposed(np.concatenate([np.diag([-1.0, 1.0, 1.0]).reshape(9), np.zeros(3)]))


def test_decomposed_jacobian_at_identity():
    from paper_1909_10690_amd.register import decomposed_jacobian
    J = decomposed_jacobian(np.zeros(12))
    gens = [np.array([[0, 0, 0], [0, 0, -1], [0, 1, 0]]),   # about x
            np.array([[0, 0, 1], [0, 0, 0], [-1, 0, 0]]),   # about y
            np.array([[0, -1, 0], [1, 0, 0], [0, 0, 0]])]   # about z
    for j, G in enumerate(gens):
        assert np.allclose(J[:9, j], G.reshape(9), atol=1e-8) and np.allclose(J[9:, j], 0, atol=1e-8)
    for j in range(3):   # log-scale j: dA = e_j e_j^T
        E = np.zeros((3, 3))
        E[j, j] = 1.0
        assert np.allclose(J[:9, 3 + j], E.reshape(9), atol=1e-8)
    shear_pos = [(0, 1), (0, 2), (1, 2)]   # h_xy, h_xz, h_yz: upper-triangular entries of A
    for j, (r, c) in enumerate(shear_pos):
        E = np.zeros((3, 3))
        E[r, c] = 1.0
        assert np.allclose(J[:9, 6 + j], E.reshape(9), atol=1e-8)
    assert np.allclose(J[9:, 9:], np.eye(3), atol=1e-8) and np.allclose(J[:9, 9:], 0, atol=1e-8)
