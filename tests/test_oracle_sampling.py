"""Pins of the oracle's random subsampling (Discussion: Mattes' MI samples
voxels at random where MI over all voxels does not; the paper leaves the
effect open).

* The counter-based generator against SplitMix64's published reference
  outputs (tests/golden/splitmix64.json).
* The keep rule written out again here, from the generator's definition,
  and the oracle's sampled histograms against exact rational brute force
  over the voxels that rule keeps.
* The kept share against the binomial law; fraction 1 (or more) against
  the full histogram; the Parzen table over the kept voxels against a
  numpy / scipy build of the same subset.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T
from tests.brute_force import hist_exact

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "splitmix64.json")
MASK64 = 2 ** 64 - 1


def splitmix64(seed: int, i: int) -> int:
    """Output i (from 0) of SplitMix64 seeded with ``seed``, in Python
    integers."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def keep_mask(shape_zyx, fraction: float, seed: int) -> np.ndarray:
    n = int(np.prod(shape_zyx))
    if fraction >= 1.0:
        return np.ones(shape_zyx, bool)
    thr = int(np.floor(fraction * 2.0 ** 32))
    return np.array([(splitmix64(seed, i) >> 32) < thr for i in range(n)]).reshape(shape_zyx)


def test_generator_matches_reference_outputs():
    for case in json.load(open(GOLDEN))["cases"]:
        for i, want in enumerate(case["outputs"]):
            assert oracle.splitmix64(case["seed"], i) == int(want)
            assert splitmix64(case["seed"], i) == int(want)


def test_generator_agrees_on_random_counters():
    rng = np.random.default_rng(3)
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        i = int(rng.integers(0, 2 ** 40))
        assert oracle.splitmix64(seed, i) == splitmix64(seed, i)


def _tiny(seed, shape=(5, 4, 3)):
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 16, size=shape[::-1]).astype(np.uint8)
    m = rng.integers(0, 16, size=shape[::-1]).astype(np.uint8)
    return f, m, rng


@pytest.mark.parametrize("fraction,seed", [(0.3, 1), (0.6, 99), (0.05, 2 ** 63 + 5)])
@pytest.mark.parametrize("clamp", [False, True])
def test_sampled_hist_matches_brute_force(fraction, seed, clamp):
    f, m, rng = _tiny(int(fraction * 100) + clamp)
    F, Mv = oracle.volume(f, 0, 15), oracle.volume(m, 0, 15)
    keep = keep_mask(f.shape, fraction, seed)
    mats = [T.translation((0.5, -0.25, 0.0)), T.translation((1.0, 0.0, -1.0))]
    mats += list(inputs.random_affines(rng, 4, f.shape[::-1], rot=20, trans=1.0).reshape(-1, 3, 4))
    for M in mats:
        h, n = oracle.hist_hard_sampled(F, Mv, M, 4, int(clamp), fraction, seed)
        ref, rn = hist_exact(f, m, M, 4, (0, 15), (0, 15), clamp=clamp, keep=keep)
        assert n == rn and np.array_equal(h.astype(np.int64), ref)


def test_kept_share_follows_the_binomial_law():
    shape = (64, 64, 64)
    f = np.zeros(shape, np.uint8)
    F = oracle.volume(f, 0, 255)
    N = f.size
    for fraction in (0.01, 0.1, 0.5, 0.9):
        for seed in (0, 12345):
            _, n = oracle.hist_hard_sampled(F, F, T.translation((0, 0, 0)), 2, oracle.CLAMP, fraction, seed)
            sd = np.sqrt(N * fraction * (1 - fraction))
            assert abs(n - fraction * N) < 6 * sd
    # different seeds give different samples
    _, a = oracle.hist_hard_sampled(F, F, T.translation((0, 0, 0)), 2, oracle.CLAMP, 0.5, 1)
    _, b = oracle.hist_hard_sampled(F, F, T.translation((0, 0, 0)), 2, oracle.CLAMP, 0.5, 2)
    assert a != b


def test_fraction_one_is_the_full_histogram():
    f, m, rng = _tiny(5, shape=(9, 7, 6))
    F, Mv = oracle.volume(f, 0, 15), oracle.volume(m, 0, 15)
    M = inputs.random_affines(rng, 1, f.shape[::-1])[0]
    full, n = oracle.hist_hard(F, Mv, M, 8)
    for frac in (1.0, 2.5):
        h, ns = oracle.hist_hard_sampled(F, Mv, M, 8, oracle.EXCLUDE, frac, 77)
        assert ns == n and np.array_equal(h, full)
    mi_full, ov_full, _ = oracle.eval_hard(F, Mv, M, 8, (1.0, 1.5))
    mi_s, ov_s, _ = oracle.eval_hard(F, Mv, M, 8, (1.0, 1.5), sample=(1.0, 3))
    assert np.array_equal(mi_full, mi_s) and np.array_equal(ov_full, ov_s)


@pytest.mark.parametrize("boundary", [oracle.CLAMP, oracle.EXCLUDE])
def test_sampled_parzen_table_matches_scipy_build(boundary):
    from scipy import ndimage
    from scipy.interpolate import BSpline
    basis = BSpline.basis_element([-2, -1, 0, 1, 2], extrapolate=False)
    rng = np.random.default_rng(11)
    shape = (14, 12, 10)
    lab = inputs.render_labels(shape)
    f = (inputs.intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0).astype(np.float32)
    m = (inputs.intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0).astype(np.float32)
    F, Mv = oracle.volume(f, 0.0, 1.0), oracle.volume(m, 0.1, 0.9)
    B, fraction, seed = 16, 0.35, 4242
    sel = keep_mask(f.shape, fraction, seed).reshape(-1)
    zz, yy, xx = np.meshgrid(*(np.arange(s) for s in f.shape), indexing="ij")
    X = np.stack([xx, yy, zz, np.ones_like(xx)], -1).reshape(-1, 4).astype(np.float64)
    mc = np.clip(m.astype(np.float64), 0.1, 0.9)
    for _ in range(3):
        M = inputs.random_affines(rng, 1, shape, rot=15, trans=2)[0].reshape(3, 4)
        h, n = oracle.parzen_table(F, Mv, M, B, boundary, sample=(fraction, seed))
        Y = X @ M.T
        top = np.array(shape, dtype=np.float64) - 1
        inside = np.all((Y >= 0) & (Y <= top), axis=1)
        keep = sel & (True if boundary == oracle.CLAMP else inside)
        Yc = np.clip(Y[keep], 0, top)
        v = ndimage.map_coordinates(mc, [Yc[:, 2], Yc[:, 1], Yc[:, 0]], order=1, mode="nearest")
        s = np.clip(1 + (v - 0.1) / 0.8 * (B - 4), 1, B - 3)
        fb = np.minimum(np.floor(np.clip(f.reshape(-1)[keep].astype(np.float64), 0, 1) * B), B - 1).astype(int)
        ref = np.zeros((B, B))
        k0 = np.floor(s).astype(int) - 1
        for d in range(4):
            kap = k0 + d
            np.add.at(ref, (fb, kap), np.nan_to_num(basis(kap - s)))
        assert n == keep.sum()
        np.testing.assert_allclose(h, ref, atol=1e-6)
