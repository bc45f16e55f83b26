"""Host-side transform construction (Introduction / Methodology: the affine
family of 12 degrees of freedom, applied about the fixed volume's centre;
Fig. 1: the Transform block maps fixed voxels into the moving volume),
checked on the CPU against their definitions point by point and against
closed forms.  (The composition of a physical matrix into voxel indices
belongs to the metric; the oracle's is pinned in the oracle tests.)

* The physical matrix of the centred parameterisation sends x to
  A (x - c) + c + t; the batch builder agrees with the single one, the
  torch builder of the autograd path with both, and the constant Jacobian
  d P / d (A, t) with differences of the builder and with torch autograd.
* Euler rotations are proper rotations; with no rotation and no shear the
  affine matrix is diag(scale).
* The registration parameterisation (angles, log-scales, shears, t) round
  trips, and its Jacobian at the identity has the closed-form columns: the
  rotation generators, the unit diagonal entries, the unit translations.
"""
import numpy as np
import pytest

from paper_1909_10690_amd import transforms as T


def test_centred_matrix_follows_its_definition():
    """P (x, 1) = A (x - c) + c + t for random points; batch = single."""
    rng = np.random.default_rng(11)
    A = np.stack([T.affine_matrix(rng.uniform(-30, 30, 3), rng.uniform(0.8, 1.2, 3), rng.uniform(-0.1, 0.1, 3))
                  for _ in range(8)])
    t = rng.uniform(-10, 10, (8, 3))
    c = rng.uniform(-100, 100, 3)
    Pb = T.centred_matrices(A, t, c).reshape(-1, 3, 4)
    for k in range(8):
        P = T.centred_matrix(A[k], t[k], c)
        assert np.array_equal(P, Pb[k])
        for _ in range(10):
            x = rng.uniform(-200, 200, 3)
            assert np.allclose(P[:, :3] @ x + P[:, 3], A[k] @ (x - c) + c + t[k], rtol=0, atol=1e-9)


def test_centred_jacobian_and_torch_builder():
    """The constant Jacobian d P / d (A, t) equals the difference of the
    builder at unit parameter steps (P is affine in them); the torch builder
    the autograd path uses equals the numpy one, and its autograd Jacobian
    equals the constant one."""
    import torch
    from paper_1909_10690_amd.autograd import centred_matrices
    rng = np.random.default_rng(12)
    c = rng.uniform(-50, 50, 3)
    J = T.centred_jacobian(c)
    base = T.centred_matrix(np.zeros((3, 3)), np.zeros(3), c).reshape(12)
    for p in range(12):
        e = np.zeros(12)
        e[p] = 1.0
        assert np.allclose(T.centred_matrix(e[:9], e[9:], c).reshape(12) - base, J[:, p], rtol=0, atol=1e-12)
    params = np.concatenate([np.stack([T.affine_matrix(rng.uniform(-20, 20, 3), rng.uniform(0.9, 1.1, 3))
                                       for _ in range(5)]).reshape(5, 9), rng.uniform(-5, 5, (5, 3))], axis=1)
    pt = torch.as_tensor(params)
    assert np.allclose(centred_matrices(pt, c).numpy(), T.centred_matrices(params[:, :9], params[:, 9:], c),
                       rtol=0, atol=1e-12)
    Jt = torch.autograd.functional.jacobian(lambda v: centred_matrices(v.reshape(1, 12), c).reshape(12),
                                            pt[0].clone())
    assert np.allclose(Jt.numpy(), J, rtol=0, atol=1e-12)


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


def test_decomposed_to_affine_matches_matrix_product():
    """The scalar form equals R(angles) H(shears) diag(exp(log-scales)) built
    from the 3x3 factors, with t passed through."""
    from paper_1909_10690_amd.register import decomposed_to_affine
    rng = np.random.default_rng(15)
    for _ in range(50):
        d = np.concatenate([rng.uniform(-0.6, 0.6, 3), rng.uniform(-0.2, 0.2, 3), rng.uniform(-0.2, 0.2, 3),
                            rng.uniform(-10, 10, 3)])
        A = T.affine_matrix(np.rad2deg(d[0:3]), np.exp(d[3:6]), d[6:9])
        np.testing.assert_allclose(decomposed_to_affine(d), np.concatenate([A.reshape(9), d[9:]]),
                                   rtol=0, atol=1e-14)


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


def test_decomposed_jacobian_against_differences():
    """The analytic Jacobian against central differences of
    decomposed_to_affine at random parameters."""
    from paper_1909_10690_amd.register import decomposed_jacobian, decomposed_to_affine
    rng = np.random.default_rng(15)
    h = 1e-6
    for _ in range(50):
        d = np.concatenate([rng.uniform(-0.6, 0.6, 3), rng.uniform(-0.2, 0.2, 3), rng.uniform(-0.2, 0.2, 3),
                            rng.uniform(-10, 10, 3)])
        J = decomposed_jacobian(d)
        for j in range(12):
            e = np.zeros(12)
            e[j] = h
            fd = (decomposed_to_affine(d + e) - decomposed_to_affine(d - e)) / (2 * h)
            assert np.allclose(J[:, j], fd, rtol=0, atol=1e-8), j
