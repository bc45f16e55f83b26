"""Pins of the oracle's hard-binned joint histogram (CPU only).

The histogram path has one correct answer under its integer rules (Q32
coordinates, 16-bit trilinear weights, floor binning).  The oracle's
128-bit implementation is checked against things that do not share its
arithmetic: an exact rational brute force, numpy slicing for integer
translations, numpy fancy indexing for axis permutations, closed-form
overlap counts and scipy's order-1 spline at dyadic coordinates.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T
from tests import brute_force as bf

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _vol(a, lo, hi):
    return oracle.volume(a, lo, hi)


def _fixed_bins(a, lo, hi, bins):
    u = np.clip(a.astype(np.int64), lo, hi) - lo
    return (u * bins) // (hi - lo + 1)


CASES = [
    # dtype, shape (nx, ny, nz), fixed range, moving range, bins
    (np.uint8, (4, 4, 4), (0, 255), (0, 255), 4),
    (np.uint16, (4, 4, 4), (0, 4095), (100, 3000), 8),
    (np.int16, (5, 4, 3), (-1000, 1500), (-300, 700), 2),
    (np.uint8, (5, 4, 3), (10, 200), (0, 99), 8),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_integer_translations_match_brute_force(case):
    dtype, shape, fr, mr, bins = CASES[case]
    rng = np.random.default_rng(100 + case)
    info = np.iinfo(dtype)
    fixed = inputs.random_volume(rng, shape, dtype, info.min if dtype != np.uint16 else 0, min(info.max, 4095))
    moving = inputs.random_volume(rng, shape, dtype, info.min if dtype != np.uint16 else 0, min(info.max, 4095))
    F, Mv = _vol(fixed, *fr), _vol(moving, *mr)
    for t in itertools.product(range(-3, 4), repeat=3):
        M = T.translation(t)
        h, n = oracle.hist_hard(F, Mv, M, bins)
        he, ne = bf.hist_exact(fixed, moving, M, bins, fr, mr)
        assert n == ne
        assert np.array_equal(h, he), t
        nx, ny, nz = shape
        assert n == max(0, nx - abs(t[0])) * max(0, ny - abs(t[1])) * max(0, nz - abs(t[2]))


def _rotations24():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            P = np.zeros((3, 3))
            for r in range(3):
                P[r, perm[r]] = signs[r]
            if round(np.linalg.det(P)) == 1:
                mats.append(P)
    assert len(mats) == 24
    return mats


def test_axis_rotations_permute_voxels():
    rng = np.random.default_rng(7)
    fixed = inputs.random_volume(rng, (4, 4, 4), np.uint8, 0, 255)
    moving = inputs.random_volume(rng, (4, 4, 4), np.uint8, 0, 255)
    F, Mv = _vol(fixed, 0, 255), _vol(moving, 0, 255)
    c = np.full(3, 1.5)
    zz, yy, xx = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    X = np.stack([xx, yy, zz], -1).reshape(-1, 3)
    for P in _rotations24():
        M = np.zeros((3, 4))
        M[:, :3] = P
        M[:, 3] = c - P @ c
        h, n = oracle.hist_hard(F, Mv, M, 8)
        he, _ = bf.hist_exact(fixed, moving, M, 8, (0, 255), (0, 255))
        assert np.array_equal(h, he)
        # numpy fancy indexing: the moving voxel each fixed voxel lands on
        Y = np.rint(X @ P.T + M[:, 3]).astype(int)
        fb = _fixed_bins(fixed[X[:, 2], X[:, 1], X[:, 0]], 0, 255, 8)
        mb = _fixed_bins(moving[Y[:, 2], Y[:, 1], Y[:, 0]], 0, 255, 8)
        ref = np.zeros((8, 8), dtype=np.int64)
        np.add.at(ref, (fb, mb), 1)
        assert n == 64 and np.array_equal(h, ref)


@pytest.mark.parametrize("seed", range(4))
def test_random_affines_match_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    shape = (4, 4, 4) if seed % 2 == 0 else (5, 4, 3)
    dtype = np.uint16 if seed < 2 else np.int16
    lo, hi = (0, 4095) if dtype == np.uint16 else (-2000, 2000)
    fixed = inputs.random_volume(rng, shape, dtype, lo, hi)
    moving = inputs.random_volume(rng, shape, dtype, lo, hi)
    fr, mr = (lo, hi), (lo + 100, hi - 100)   # moving values beyond the range get clamped
    F, Mv = _vol(fixed, *fr), _vol(moving, *mr)
    for _ in range(25):
        A = T.affine_matrix(rng.uniform(-40, 40, 3), rng.uniform(0.7, 1.3, 3), rng.uniform(-0.2, 0.2, 3))
        M = T.centred_matrix(A, rng.uniform(-1.5, 1.5, 3), T.fixed_centre(shape))
        for clamp in (False, True):
            h, n = oracle.hist_hard(F, Mv, M, 8, oracle.CLAMP if clamp else oracle.EXCLUDE)
            he, ne = bf.hist_exact(fixed, moving, M, 8, fr, mr, clamp=clamp)
            assert n == ne and np.array_equal(h, he)
            if clamp:
                assert n == fixed.size


def test_integer_translation_equals_histogram2d_of_slices():
    c = inputs.plain_translation(n=32, seed=5)
    f, m = c["fixed"], c["moving"]
    F, Mv = _vol(f, 0, 255), _vol(m, 0, 255)
    for t in [(0, 0, 0), (3, -2, 1), (-7, 5, 0), (31, 0, 0), (32, 0, 0), (-5, -5, -5)]:
        h, n = oracle.hist_hard(F, Mv, T.translation(t), 32)
        tx, ty, tz = t
        fs = f[max(0, -tz):32 - max(0, tz), max(0, -ty):32 - max(0, ty), max(0, -tx):32 - max(0, tx)]
        ms = m[max(0, tz):32 + min(0, tz), max(0, ty):32 + min(0, ty), max(0, tx):32 + min(0, tx)]
        ref, _, _ = np.histogram2d(fs.ravel().astype(float), ms.ravel().astype(float), bins=32,
                                   range=[[0, 256], [0, 256]])
        assert n == fs.size
        assert np.array_equal(h, ref.astype(np.int64)), t


def test_half_voxel_shift_is_mean_of_neighbours():
    rng = np.random.default_rng(9)
    fixed = inputs.random_volume(rng, (9, 3, 2), np.uint16, 0, 65535)
    moving = inputs.random_volume(rng, (9, 3, 2), np.uint16, 0, 65535)
    F, Mv = _vol(fixed, 0, 65535), _vol(moving, 0, 65535)
    bins = 256
    h, n = oracle.hist_hard(F, Mv, T.translation((0.5, 0, 0)), bins)
    # value = (v_i + v_{i+1}) / 2 exactly; bin = floor(value * B / R)
    s = moving[:, :, :-1].astype(np.int64) + moving[:, :, 1:].astype(np.int64)
    mb = (s * bins) // (2 * 65536)
    fb = _fixed_bins(fixed[:, :, :-1], 0, 65535, bins)
    ref = np.zeros((bins, bins), dtype=np.int64)
    np.add.at(ref, (fb.ravel(), mb.ravel()), 1)
    assert n == 8 * 3 * 2 and np.array_equal(h, ref)


def test_quarter_voxel_coordinates_match_scipy_trilinear():
    """Coordinates on a 1/4-voxel lattice make the 16-bit weights exact, so
    the oracle's bins equal those of scipy's order-1 spline values."""
    from scipy import ndimage
    rng = np.random.default_rng(11)
    shape = (12, 10, 8)
    fixed = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    moving = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    F, Mv = _vol(fixed, 0, 255), _vol(moving, 0, 255)
    zz, yy, xx = np.meshgrid(*(np.arange(s) for s in shape[::-1]), indexing="ij")
    X = np.stack([xx, yy, zz, np.ones_like(xx)], -1).reshape(-1, 4).astype(np.float64)
    for _ in range(20):
        M = np.zeros((3, 4))
        M[:, :3] = rng.integers(-4, 5, (3, 3)) / 4.0
        M[:, 3] = rng.integers(-8, 40, 3) / 4.0
        h, n = oracle.hist_hard(F, Mv, M, 16)
        Y = X @ M.T
        inside = np.all((Y >= 0) & (Y <= np.array(shape) - 1), axis=1)
        vals = ndimage.map_coordinates(moving.astype(np.float64), [Y[inside, 2], Y[inside, 1], Y[inside, 0]], order=1)
        mb = np.floor(vals * 16 / 256).astype(np.int64)
        fb = _fixed_bins(fixed.reshape(-1)[inside], 0, 255, 16)
        ref = np.zeros((16, 16), dtype=np.int64)
        np.add.at(ref, (fb, mb), 1)
        assert n == inside.sum() and np.array_equal(h, ref)


def test_identity_counts_every_voxel_and_diagonal():
    c = inputs.plain_translation(n=24, seed=3)
    F = _vol(c["fixed"], 0, 255)
    h, n = oracle.hist_hard(F, F, T.translation((0, 0, 0)), 32)
    assert n == 24 ** 3
    assert np.array_equal(np.diag(np.diag(h)), h)
    assert np.array_equal(np.diag(h), np.bincount(c["fixed"].ravel() >> 3, minlength=32))


def test_quantize_round_half_even_and_limits():
    Mq, st = oracle.quantize(np.array([1, 0, 0, 2 ** -33, 0, 1, 0, 3 * 2 ** -33, 0, 0, 1, -2 ** -33]))
    assert st == 0
    assert Mq[0] == 2 ** 32 and Mq[3] == 0 and Mq[7] == 2 and Mq[11] == 0
    for bad in (np.nan, np.inf, 65536.5):
        M = T.translation((0, 0, 0)).reshape(12)
        M[1] = bad
        assert oracle.quantize(M)[1] == 1
    M = T.translation((2 ** 24 + 1, 0, 0))
    assert oracle.quantize(M)[1] == 1
    assert oracle.quantize(T.translation((2 ** 24, 0, 0)))[1] == 0


def test_unusable_transform_gives_nan_and_empty():
    rng = np.random.default_rng(1)
    v = inputs.random_volume(rng, (4, 4, 4), np.uint8, 0, 255)
    F = _vol(v, 0, 255)
    M = np.stack([T.translation((0, 0, 0)), T.translation((np.nan, 0, 0))]).reshape(2, 12)
    mi, ov, hist = oracle.eval_hard(F, F, M, 4, [1.0, 2.0], want_hist=True)
    assert np.all(np.isnan(mi[1])) and ov[1] == 0 and hist[1].sum() == 0
    assert np.isfinite(mi[0]).all() and ov[0] == 64


def test_zero_overlap_gives_zero():
    rng = np.random.default_rng(2)
    v = inputs.random_volume(rng, (6, 5, 4), np.uint8, 0, 255)
    F = _vol(v, 0, 255)
    mi, ov, _ = oracle.eval_hard(F, F, T.translation((100, 0, 0)), 8, [1.0, 0.5, 2.0])
    assert ov[0] == 0 and np.all(mi == 0.0)


def test_full_range_u16_extremes():
    """R = 65536: V reaches (2^16 - 1) * 2^48 and the top value maps to B-1."""
    fixed = np.full((2, 2, 3), 65535, dtype=np.uint16)
    fixed[0, 0, 0] = 0
    F = _vol(fixed, 0, 65535)
    h, n = oracle.hist_hard(F, F, T.translation((0.999, 0, 0)), 256)
    he, ne = bf.hist_exact(fixed, fixed, T.translation((0.999, 0, 0)), 256, (0, 65535), (0, 65535))
    assert n == ne == 8 and np.array_equal(h, he)
    assert h[255].sum() >= 1
