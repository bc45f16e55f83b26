"""Host-side construction of the parameter-space maps (Results: the
translation, rotation and scale grids), checked on the CPU against
properties fixed by the mathematics rather than by the code under test.

* Z order is a permutation of the grid rows, and for a power-of-two edge
  each run of 8 consecutive rows is a 2x2x2 block of the grid.
* Versor rotations are proper rotations (orthonormal, det +1) and equal the
  Rodrigues rotation by 2 asin|p| about p / |p|; vectors outside the unit
  sphere give the rotation by 180 degrees about their direction.
* Grid rows are x-parameter fastest; the families' matrices are x + p,
  diag(1 + p) and the rotation; the grid centre is the identity map.
"""
import numpy as np
import pytest

from paper_1909_10690_amd import maps


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 51])
def test_z_order_is_a_permutation(n):
    o = maps.z_order(n)
    assert o.shape == (n ** 3,)
    assert np.array_equal(np.sort(o), np.arange(n ** 3))


@pytest.mark.parametrize("n", [2, 4, 8])
def test_z_order_runs_of_eight_are_cubes(n):
    o = maps.z_order(n)
    k, r = np.divmod(o, n * n)
    j, i = np.divmod(r, n)
    for s in range(0, n ** 3, 8):
        for axis in (i[s:s + 8], j[s:s + 8], k[s:s + 8]):
            assert axis.max() - axis.min() == 1 and axis.min() % 2 == 0


def rodrigues(axis, angle):
    """Rotation by `angle` about the unit vector `axis` (Rodrigues' formula)."""
    kx, ky, kz = axis
    K = np.array([[0.0, -kz, ky], [kz, 0.0, -kx], [-ky, kx, 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def test_versors_are_rodrigues_rotations():
    rng = np.random.default_rng(7)
    v = rng.uniform(-1, 1, (400, 3))
    v = v[np.linalg.norm(v, axis=1) <= 1.0]
    R = maps.versor_matrices(v)
    for Ri, vi in zip(R, v):
        assert np.allclose(Ri @ Ri.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(Ri) - 1.0) < 1e-12
        s = np.linalg.norm(vi)
        if s < 1e-9:
            assert np.allclose(Ri, np.eye(3), atol=1e-12)
            continue
        assert np.allclose(Ri, rodrigues(vi / s, 2.0 * np.arcsin(s)), atol=1e-12)


def test_versors_outside_the_unit_sphere_turn_half_way():
    v = np.array([[2.0, 0.0, 0.0], [0.0, -3.0, 0.0], [1.0, 1.0, 1.0], [0.9, 0.9, 0.0]])
    R = maps.versor_matrices(v)
    for Ri, vi in zip(R, v):
        a = vi / np.linalg.norm(vi)
        assert np.allclose(Ri, rodrigues(a, np.pi), atol=1e-12)
        assert abs(np.trace(Ri) + 1.0) < 1e-12  # 180 degrees: trace 1 + 2 cos(pi)


def test_grid_rows_x_fastest_and_centred():
    n, ext = 5, 2.0
    g = maps.grid_axis(n, ext)
    assert np.allclose(g, [-2.0, -1.0, 0.0, 1.0, 2.0])
    p = maps.grid_params(n, ext)
    for (i, j, k) in [(0, 0, 0), (4, 0, 0), (1, 3, 2), (4, 4, 4)]:
        assert np.array_equal(p[(k * n + j) * n + i], [g[i], g[j], g[k]])
    assert np.array_equal(maps.grid_axis(1, 3.0), [0.0])
    with pytest.raises(ValueError):
        maps.grid_axis(0, 1.0)


def test_family_matrices():
    p = np.array([[0.5, -1.0, 2.0], [0.0, 0.0, 0.0]])
    A, t = maps.family_affines("translation", p)
    assert np.array_equal(A, np.broadcast_to(np.eye(3), (2, 3, 3))) and np.array_equal(t, p)
    A, t = maps.family_affines("scale", p)
    assert np.allclose(A[0], np.diag([1.5, 0.0, 3.0])) and not t.any()
    A, t = maps.family_affines("rotation", p[1:])
    assert np.allclose(A[0], np.eye(3)) and not t.any()
    with pytest.raises(ValueError):
        maps.family_affines("shear", p)


@pytest.mark.parametrize("family", maps.FAMILIES)
def test_grid_centre_is_the_identity_map(family):
    n = 5
    M = maps.map_transforms(family, n, (16, 12, 9))
    centre = M[(2 * n + 2) * n + 2].reshape(3, 4)
    assert np.allclose(centre, np.hstack([np.eye(3), np.zeros((3, 1))]), atol=1e-12)
    # a grid point off the centre is not the identity
    assert not np.allclose(M[0].reshape(3, 4), centre)
