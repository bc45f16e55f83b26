"""Seeded synthetic workloads (stand-ins for the paper's HCP volumes),
checked on the CPU for the properties their recipes state.

* The resampler that builds moving volumes under a known transform is
  trilinear: interior samples equal a hand-written trilinear interpolation
  (to 5e-4 on values up to 100: the resampler maps coordinates in fp32,
  under 1e-6 voxel of error here).
* ``invert`` inverts a 3x4 affine map.
* Generators are deterministic in their seed; the uneven pairs do not depend
  on the number of threads that build them.
* The multi-modal sweep's grid covers tx x rot_z x scale as stated; volumes
  stay in their declared ranges and dtypes.
"""
import numpy as np

from paper_1909_10690_amd import inputs, transforms as T


def trilinear(vol, p):
    """vol (z, y, x) at the continuous point p = (x, y, z), p inside."""
    x, y, z = p
    x0, y0, z0 = int(np.floor(x)), int(np.floor(y)), int(np.floor(z))
    fx, fy, fz = x - x0, y - y0, z - z0
    acc = 0.0
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (fx if dx else 1 - fx) * (fy if dy else 1 - fy) * (fz if dz else 1 - fz)
                acc += w * float(vol[z0 + dz, y0 + dy, x0 + dx])
    return acc


def test_resampler_is_trilinear():
    rng = np.random.default_rng(21)
    vol = rng.uniform(0, 100, (9, 11, 13))
    A = T.affine_matrix((5.0, -3.0, 8.0), (1.05, 0.97, 1.0))
    M = T.centred_matrix(A, (0.7, -0.4, 0.3), T.fixed_centre((13, 11, 9)))   # fixed index -> moving index
    out = inputs.resample_trilinear(vol, M)                 # out[i] = vol(M^-1 i)
    Mi = inputs.invert(M)
    checked = 0
    for _ in range(200):
        i = np.array([rng.integers(0, 13), rng.integers(0, 11), rng.integers(0, 9)], dtype=np.float64)
        p = Mi[:, :3] @ i + Mi[:, 3]
        if np.all(p >= 0) and np.all(p < np.array([12, 10, 8])):
            assert abs(out[int(i[2]), int(i[1]), int(i[0])] - trilinear(vol, p)) < 5e-4
            checked += 1
    assert checked > 50


def test_invert_composes_to_identity():
    rng = np.random.default_rng(22)
    for _ in range(20):
        M = T.centred_matrix(T.affine_matrix(rng.uniform(-30, 30, 3), rng.uniform(0.8, 1.2, 3)),
                           rng.uniform(-5, 5, 3), (20, 30, 40))
        Mi = inputs.invert(M)
        p = rng.uniform(-10, 50, 3)
        q = M[:, :3] @ p + M[:, 3]
        assert np.allclose(Mi[:, :3] @ q + Mi[:, 3], p, atol=1e-10)


def test_generators_are_deterministic():
    a, b = inputs.plain_translation(), inputs.plain_translation()
    assert np.array_equal(a["fixed"], b["fixed"]) and np.array_equal(a["moving"], b["moving"])
    assert a["fixed"].dtype == np.uint8 and a["fixed"].shape == (64, 64, 64)
    assert a["transforms"].shape == (21, 12) and np.allclose(a["transforms"][:, 3], np.arange(-10, 11))
    c = inputs.plain_translation(seed=1)
    assert not np.array_equal(a["fixed"], c["fixed"])


def test_multimodal_grid_and_ranges():
    w = inputs.multimodal_sweep(shape_xyz=(24, 20, 12))
    assert w["transforms"].shape == (1000, 12)
    assert w["fixed"].dtype == np.uint16 and w["fixed"].max() <= 4095
    assert w["moving"].dtype == np.uint16 and w["moving"].max() <= 4095
    assert w["q"] == [1.0, 0.5, 0.8, 1.2, 1.5, 2.0] and w["bins"] == 128
    # first and last grid points: tx -10, rot_z -15 deg, scale 0.9 / tx 10, rot_z 15, scale 1.1
    first = T.centred_matrix(T.affine_matrix((0, 0, -15.0), 0.9), (-10.0, 0, 0), T.fixed_centre((24, 20, 12))).reshape(12)
    last = T.centred_matrix(T.affine_matrix((0, 0, 15.0), 1.1), (10.0, 0, 0), T.fixed_centre((24, 20, 12))).reshape(12)
    assert np.allclose(w["transforms"][0], first) and np.allclose(w["transforms"][-1], last)


def test_uneven_pairs_independent_of_threads():
    p1 = inputs.uneven_pairs(n_pairs=5, edges=(8, 12, 16), threads=1)
    p4 = inputs.uneven_pairs(n_pairs=5, edges=(8, 12, 16), threads=4)
    for a, b in zip(p1, p4):
        assert np.array_equal(a["fixed"], b["fixed"]) and np.array_equal(a["moving"], b["moving"])
        assert np.array_equal(a["transforms"], b["transforms"])
        assert a["transforms"].shape == (16, 12) and a["fixed"].dtype == np.uint8
        assert all(e in (8, 12, 16) for e in a["fixed"].shape)


def test_random_volume_range_and_dtype():
    rng = np.random.default_rng(23)
    v = inputs.random_volume(rng, (7, 5, 3), np.int16, -1000, 1500)
    assert v.shape == (3, 5, 7) and v.dtype == np.int16 and v.min() >= -1000 and v.max() <= 1500
    f = inputs.random_volume(rng, (4, 4, 4), np.float32, 0.0, 1.0)
    assert f.dtype == np.float32 and 0.0 <= f.min() and f.max() <= 1.0
