"""Pins of the oracle's Parzen (cubic B-spline) joint table and its gradient.

The Parzen-windowed histogram is the differentiable variant of the joint
histogram (the windowed-histogram idea behind the Mattes metric the paper
compares against, Methodology and Discussion).  Pinned against scipy's
B-spline basis and order-1 spline, the partition of unity, and central
finite differences of the oracle's own forward pass (which exercises the
analytic gradient's every term: a dropped term, sign or transposed index
shows up as a mismatch).
"""
import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T


def _bspline():
    from scipy.interpolate import BSpline
    return BSpline.basis_element(np.arange(-2.0, 3.0), extrapolate=False)


def test_beta3_matches_scipy_basis():
    b = _bspline()
    db = b.derivative()
    for t in np.linspace(-2.5, 2.5, 1001):
        ref = 0.0 if abs(t) >= 2 else float(b(t))
        dref = 0.0 if abs(t) >= 2 else float(db(t))
        assert abs(oracle.beta3(t) - ref) < 1e-15
        assert abs(oracle.dbeta3(t) - dref) < 1e-14


def _case(seed=0, shape=(20, 18, 16), dtype=np.float32):
    rng = np.random.default_rng(seed)
    lab = inputs.render_labels(shape)
    f = inputs.intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0
    truth = T.centred_matrix(T.affine_matrix((4, -3, 6), 1.02), (1.2, -0.8, 0.5), T.fixed_centre(shape))
    lab_m = inputs.render_labels(shape, inv_map=inputs.invert(truth))
    m = inputs.intensities(lab_m, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0
    return f.astype(dtype), m.astype(dtype), rng


@pytest.mark.parametrize("boundary", [oracle.CLAMP, oracle.EXCLUDE])
def test_table_matches_scipy_build(boundary):
    from scipy import ndimage
    f, m, rng = _case()
    shape = f.shape[::-1]
    F, Mv = oracle.volume(f, 0.0, 1.0), oracle.volume(m, 0.1, 0.9)
    B = 16
    basis = _bspline()
    zz, yy, xx = np.meshgrid(*(np.arange(s) for s in f.shape), indexing="ij")
    X = np.stack([xx, yy, zz, np.ones_like(xx)], -1).reshape(-1, 4).astype(np.float64)
    mc = np.clip(m.astype(np.float64), 0.1, 0.9)
    for _ in range(4):
        M = inputs.random_affines(rng, 1, shape, rot=15, trans=3)[0].reshape(3, 4)
        h, n = oracle.parzen_table(F, Mv, M, B, boundary)
        Y = X @ M.T
        top = np.array(shape, dtype=np.float64) - 1
        inside = np.all((Y >= 0) & (Y <= top), axis=1)
        keep = np.ones(len(Y), bool) if boundary == oracle.CLAMP else inside
        Yc = np.clip(Y[keep], 0, top)
        v = ndimage.map_coordinates(mc, [Yc[:, 2], Yc[:, 1], Yc[:, 0]], order=1, mode="nearest")
        s = np.clip(1 + (v - 0.1) / 0.8 * (B - 4), 1, B - 3)
        fb = np.minimum(np.floor(np.clip(f.reshape(-1)[keep].astype(np.float64), 0, 1) * B), B - 1).astype(int)
        ref = np.zeros((B, B))
        k0 = np.floor(s).astype(int) - 1
        for d in range(4):
            kap = k0 + d
            w = np.nan_to_num(basis(kap - s))
            np.add.at(ref, (fb, kap), w)
        assert n == keep.sum()
        np.testing.assert_allclose(h, ref, atol=1e-6)
        assert abs(h.sum() - n) < 1e-9 * n   # partition of unity


@pytest.mark.parametrize("form", [oracle.ADDITIVE, oracle.PSEUDOADDITIVE])
def test_gradient_matches_finite_differences(form):
    f, m, rng = _case(seed=1, shape=(28, 26, 24))
    shape = f.shape[::-1]
    F, Mv = oracle.volume(f, 0.0, 1.0), oracle.volume(m, 0.0, 1.0)
    qs = [1.0, 1.5, 0.7]
    B = 16
    # finite differences on the translation column use a unit lever arm;
    # linear entries multiply voxel indices up to ~27, so their step is
    # scaled down to keep the displacement comparable
    for M in inputs.random_affines(rng, 2, shape, rot=8, trans=3):
        mi, g = oracle.parzen_grad(F, Mv, M, B, qs, oracle.CLAMP, form)
        for e, step in [(3, 1e-3), (7, 1e-3), (11, 1e-3), (0, 5e-5), (5, 5e-5), (9, 5e-5), (2, 5e-5)]:
            Mp, Mm = M.copy(), M.copy()
            Mp[e] += step
            Mm[e] -= step
            a, _ = oracle.eval_parzen(F, Mv, Mp, B, qs, oracle.CLAMP, form)
            b, _ = oracle.eval_parzen(F, Mv, Mm, B, qs, oracle.CLAMP, form)
            fd = (a[0] - b[0]) / (2 * step)
            scale = np.abs(g[0]).max(axis=1)
            assert np.all(np.abs(g[0][:, e] - fd) <= 1e-2 * scale), (e, g[0][:, e], fd)


def test_gradient_centred_params_chain_rule():
    """d MI / d(A, t) = J^T d MI / dM with the constant Jacobian of the
    centred parameterisation, checked by finite differences in (A, t)."""
    f, m, rng = _case(seed=2, shape=(24, 24, 20))
    shape = f.shape[::-1]
    F, Mv = oracle.volume(f, 0.0, 1.0), oracle.volume(m, 0.0, 1.0)
    c = T.fixed_centre(shape)
    J = T.centred_jacobian(c)
    A = T.affine_matrix((3, -2, 5), (1.01, 0.99, 1.0))
    t = np.array([0.7, -1.1, 0.4])
    p0 = T.params_from(A, t)
    M0 = T.centred_matrix(A, t, c).reshape(12)
    assert np.allclose(J @ p0 + T.centred_matrix(np.zeros((3, 3)), np.zeros(3), c).reshape(12), M0)
    mi, gM = oracle.parzen_grad(F, Mv, M0, 16, [1.0])
    gp = J.T @ gM[0, 0]
    for p, step in [(9, 1e-3), (10, 1e-3), (11, 1e-3), (0, 1e-4), (4, 1e-4), (1, 1e-4)]:
        pp, pm = p0.copy(), p0.copy()
        pp[p] += step
        pm[p] -= step
        a, _ = oracle.eval_parzen(F, Mv, T.centred_matrix(pp[:9], pp[9:], c), 16, [1.0])
        b, _ = oracle.eval_parzen(F, Mv, T.centred_matrix(pm[:9], pm[9:], c), 16, [1.0])
        fd = (a[0, 0] - b[0, 0]) / (2 * step)
        assert abs(gp[p] - fd) <= 1e-2 * np.abs(gp).max(), (p, gp[p], fd)


def test_unusable_and_empty():
    f, m, _ = _case()
    F, Mv = oracle.volume(f, 0.0, 1.0), oracle.volume(m, 0.0, 1.0)
    M = np.stack([T.translation((np.inf, 0, 0)), T.translation((500, 0, 0))]).reshape(2, 12)
    mi, g = oracle.parzen_grad(F, Mv, M, 16, [1.0, 2.0], oracle.EXCLUDE)
    assert np.all(np.isnan(mi[0])) and np.all(g[0] == 0)
    assert np.all(mi[1] == 0) and np.all(g[1] == 0)


def test_integer_fixed_dtype_bins():
    """Integer fixed volumes use the integer bin rule in the Parzen path too."""
    rng = np.random.default_rng(3)
    f = inputs.random_volume(rng, (6, 5, 4), np.uint8, 0, 255)
    m = inputs.random_volume(rng, (6, 5, 4), np.uint16, 0, 4095)
    F, Mv = oracle.volume(f, 0, 255), oracle.volume(m, 0, 4095)
    h, n = oracle.parzen_table(F, Mv, T.translation((0, 0, 0)), 8)
    rows = np.bincount((f.ravel().astype(int) * 8) // 256, minlength=8)
    np.testing.assert_allclose(h.sum(axis=1), rows, rtol=1e-12)
