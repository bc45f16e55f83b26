"""GPU parity of the hard-binned path (mi_eval through the C ABI) against
the CPU oracle: joint histograms bit-exact, overlap counts exact, MI within
1e-12 * max(1, |MI|) for Shannon and every Tsallis q."""
import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T

pytestmark = pytest.mark.gpu

MI_TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1909_10690_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    c.close()


def run_gpu(ctx, fixed, moving, frange, mrange, mats, bins, q, flags=0):
    import torch
    from paper_1909_10690_amd import binding as B
    F = B.Volume.from_numpy(fixed, *frange)
    Mv = B.Volume.from_numpy(moving, *mrange)
    tr = torch.from_numpy(np.ascontiguousarray(np.asarray(mats, dtype=np.float64).reshape(-1, 12))).cuda()
    mi, ov, hist = ctx.eval(F, Mv, tr, bins, q, flags=flags, want_hist=True)
    torch.cuda.synchronize()
    return mi.cpu().numpy(), ov.cpu().numpy(), hist.cpu().numpy().astype(np.uint32)


def run_oracle(fixed, moving, frange, mrange, mats, bins, q, flags=0):
    F = oracle.volume(fixed, *frange)
    Mv = oracle.volume(moving, *mrange)
    return oracle.eval_hard(F, Mv, mats, bins, q, boundary=flags & 1,
                            form=oracle.PSEUDOADDITIVE if flags & 0x10 else oracle.ADDITIVE,
                            want_hist=True)


def assert_parity(g, o, label=""):
    gmi, gov, gh = g
    omi, oov, oh = o
    assert np.array_equal(gov.astype(np.int64), oov), label
    for t in range(len(oov)):
        assert np.array_equal(gh[t], oh[t]), f"{label} histogram of transform {t}"
    nan = np.isnan(omi)
    assert np.array_equal(np.isnan(gmi), nan), label
    err = np.abs(gmi[~nan] - omi[~nan]) / np.maximum(1.0, np.abs(omi[~nan]))
    assert err.size == 0 or err.max() <= MI_TOL, f"{label} max rel err {err.max()}"


@pytest.mark.parametrize("flags", [0, 1, 0x10])
def test_plain_translation_sweep(ctx, flags):
    c = inputs.plain_translation()
    q = [1.0, 0.5, 2.0, 1.3]
    args = (c["fixed"], c["moving"], c["fixed_range"], c["moving_range"], c["transforms"], c["bins"], q, flags)
    g = run_gpu(ctx, *args)
    o = run_oracle(*args)
    assert_parity(g, o, f"flags={flags}")
    assert int(np.argmax(g[0][:, 0])) - 10 in (3, 4)


CASES = [
    # dtype fixed, dtype moving, shape fixed (nx,ny,nz), shape moving, frange, mrange, bins
    (np.uint8, np.uint8, (67, 45, 33), (61, 50, 29), (0, 255), (0, 255), 32),
    (np.uint16, np.uint16, (40, 36, 30), (44, 30, 33), (0, 4095), (0, 4095), 128),
    (np.int16, np.int16, (33, 35, 31), (30, 40, 32), (-1000, 1500), (-1000, 1500), 100),
    (np.uint16, np.uint8, (50, 17, 9), (70, 13, 21), (0, 65535), (0, 255), 7),
    (np.uint8, np.uint16, (31, 29, 27), (32, 28, 26), (10, 200), (0, 65535), 256),
    (np.int16, np.uint16, (64, 20, 10), (65, 21, 11), (-32768, 32767), (300, 2999), 129),
    (np.float32, np.int16, (37, 21, 19), (36, 22, 18), (0.0, 1.0), (-200, 200), 200),
    (np.uint8, np.uint8, (2, 2, 2), (2, 2, 2), (0, 255), (0, 255), 2),
    (np.uint8, np.uint8, (130, 3, 2), (129, 2, 3), (0, 255), (0, 255), 64),
]


def _random_case(case, seed):
    fd, md, fs, ms, fr, mr, bins = CASES[case]
    rng = np.random.default_rng(1000 + 17 * case + seed)

    def vol(dtype, shape, r):
        if np.dtype(dtype).kind == "f":
            return inputs.random_volume(rng, shape, dtype, -0.2, 1.2)
        info = np.iinfo(dtype)
        return inputs.random_volume(rng, shape, dtype, max(info.min, int(r[0]) - 50), min(info.max, int(r[1]) + 50))

    fixed, moving = vol(fd, fs, fr), vol(md, ms, mr)
    mats = [T.translation((0, 0, 0)), T.translation((1, -1, 0)), T.translation((0.5, 0.25, -0.75))]
    for _ in range(13):
        A = T.affine_matrix(rng.uniform(-40, 40, 3), rng.uniform(0.7, 1.3, 3), rng.uniform(-0.2, 0.2, 3))
        mats.append(T.centred_matrix(A, rng.uniform(-6, 6, 3), T.fixed_centre(fs)))
    return fixed, moving, fr, mr, np.stack(mats).reshape(-1, 12), bins


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("flags", [0, 1])
def test_random_affines(ctx, case, flags):
    fixed, moving, fr, mr, mats, bins = _random_case(case, flags)
    q = [1.0, 0.5, 0.8, 1.2, 1.5, 2.0]
    assert_parity(run_gpu(ctx, fixed, moving, fr, mr, mats, bins, q, flags),
                  run_oracle(fixed, moving, fr, mr, mats, bins, q, flags), f"case {case}")


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("boundary", [0, 1])
def test_compact_slabs_hint(ctx, case, boundary):
    """Bricks instead of thin slabs (MI_COMPACT_SLABS): the same exact
    histograms, on every shape including ragged row groups and slices."""
    from paper_1909_10690_amd import binding as B
    fixed, moving, fr, mr, mats, bins = _random_case(case, 7 + boundary)
    q = [1.0, 1.5]
    print(f"compact slabs case {case} boundary {boundary}", flush=True)
    g = run_gpu(ctx, fixed, moving, fr, mr, mats, bins, q, boundary | B.COMPACT_SLABS)
    assert_parity(g, run_oracle(fixed, moving, fr, mr, mats, bins, q, boundary), f"case {case}")


def test_compact_slabs_rotation_map(ctx):
    """A rotation map of the same image with and without the hint (the maps
    module sets it for rotations): identical MI maps."""
    import torch
    from paper_1909_10690_amd import binding as B
    from paper_1909_10690_amd import maps
    c = inputs.same_image((48, 40, 36), seed=2, dtype=np.uint16)
    F = B.Volume.from_numpy(c["fixed"], *c["fixed_range"])
    tr = torch.from_numpy(maps.map_transforms("rotation", 9, (48, 40, 36))).cuda()
    a, _, ha = ctx.eval(F, F, tr, 128, (1.0, 2.0), want_hist=True)
    b, _, hb = ctx.eval(F, F, tr, 128, (1.0, 2.0), flags=B.COMPACT_SLABS, want_hist=True)
    m = maps.mi_map(ctx, F, F, "rotation", 9, bins=128, q=(1.0, 2.0), batch=100)
    torch.cuda.synchronize()
    assert torch.equal(ha, hb) and torch.equal(a, b)
    # batches of 100 may slice the reduction differently: last bits only
    ref = a.t().reshape(2, 9, 9, 9)
    assert torch.all((m - ref).abs() <= 1e-12 * torch.clamp(ref.abs(), min=1.0))


@pytest.mark.parametrize("n,shape", [(300, (40, 36, 30)), (5000, (12, 10, 9))])
def test_processing_order_keeps_histograms(ctx, n, shape):
    """Batches of 64 transforms or more are swept in an order that groups
    similar moving depths (sorted per block of 4096 transforms): every
    transform's histogram, MI and overlap equal those of the same transform
    evaluated in batches of 50, which keep the batch order.  The affines
    turn about every axis and scale along z, so the order differs from the
    batch order; n = 5000 spans two sorted blocks."""
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(404)
    f = inputs.random_volume(rng, shape, np.uint16, 0, 4095)
    m = inputs.random_volume(rng, shape, np.uint16, 0, 4095)
    mats = inputs.random_affines(rng, n, shape, rot=25.0, trans=4.0, scale=(0.8, 1.25))
    F, Mv = B.Volume.from_numpy(f, 0, 4095), B.Volume.from_numpy(m, 0, 4095)
    q = (1.0, 1.5)
    print(f"processing order n={n} shape={shape}", flush=True)
    mi, ov, hist = ctx.eval(F, Mv, torch.from_numpy(mats).cuda(), 32, q, want_hist=True)
    torch.cuda.synchronize()
    for t0 in range(0, n, 50):
        sub = torch.from_numpy(mats[t0:t0 + 50]).cuda()
        mi_s, ov_s, h_s = ctx.eval(F, Mv, sub, 32, q, want_hist=True)
        torch.cuda.synchronize()
        assert torch.equal(hist[t0:t0 + 50], h_s), f"histograms of transforms {t0}..{t0 + 49}"
        assert torch.equal(ov[t0:t0 + 50], ov_s)
        # the reduction slices a batch of 50 and one of n differently: last bits
        assert torch.all((mi[t0:t0 + 50] - mi_s).abs() <= 1e-12 * torch.clamp(mi_s.abs(), min=1.0))


def test_integer_translations_tiny(ctx):
    import itertools
    rng = np.random.default_rng(5)
    fixed = inputs.random_volume(rng, (4, 4, 4), np.uint16, 0, 4095)
    moving = inputs.random_volume(rng, (4, 4, 4), np.uint16, 0, 4095)
    mats = np.stack([T.translation(t) for t in itertools.product(range(-4, 5), repeat=3)]).reshape(-1, 12)
    args = (fixed, moving, (0, 4095), (100, 3000), mats, 8, [1.0, 2.0])
    assert_parity(run_gpu(ctx, *args), run_oracle(*args), "4^3 translations")


def test_degenerate_transforms(ctx):
    rng = np.random.default_rng(6)
    fixed = inputs.random_volume(rng, (20, 18, 16), np.uint8, 0, 255)
    moving = inputs.random_volume(rng, (21, 17, 15), np.uint8, 0, 255)
    mats = [T.translation((0, 0, 0)), T.translation((np.nan, 0, 0)), T.translation((1000, 0, 0)),
            T.translation((2 ** 24 + 1, 0, 0)), T.translation((-21, 0, 0)), T.translation((20, 16, 14)),
            np.array([[70000.0, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]]), np.zeros((3, 4)),
            T.translation((np.inf, 0, 0))]
    mats = np.stack(mats).reshape(-1, 12)
    for flags in (0, 1):
        args = (fixed, moving, (0, 255), (0, 255), mats, 16, [1.0, 0.7], flags)
        g, o = run_gpu(ctx, *args), run_oracle(*args)
        assert_parity(g, o, f"degenerate flags={flags}")
        assert np.all(np.isnan(g[0][[1, 3, 6, 8]]))
        if flags == 0:
            assert g[1][2] == 0 and np.all(g[0][2] == 0)


def test_no_transforms(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    v = B.Volume(torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda"), 0, 255)
    mi, ov, _ = ctx.eval(v, v, torch.zeros((0, 12), dtype=torch.float64, device="cuda"), 8, [1.0])
    assert mi.shape == (0, 1)


def test_deterministic_and_self_information(ctx):
    from scipy.stats import entropy
    c = inputs.multimodal_sweep(shape_xyz=(96, 80, 40), n_tx=3, n_rot=3, n_scale=3)
    args = (c["fixed"], c["moving"], c["fixed_range"], c["moving_range"], c["transforms"], c["bins"], c["q"])
    a, b = run_gpu(ctx, *args), run_gpu(ctx, *args)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[0], b[0])
    ident = T.translation((0, 0, 0))
    g = run_gpu(ctx, c["fixed"], c["fixed"], (0, 4095), (0, 4095), ident, 128, [1.0])
    counts = np.bincount((c["fixed"].ravel().astype(np.int64) * 128) // 4096, minlength=128)
    assert abs(g[0][0, 0] - entropy(counts.astype(float))) <= 1e-12 * 5


def test_multimodal_sweep_full_size_sampled(ctx):
    """The benchmark's launch: 1000 transforms over 256x256x180 u16, 128
    bins, 6 entropies.  Sampled transforms against the oracle; every
    transform checked for mass == overlap and Shannon MI >= 0."""
    c = inputs.multimodal_sweep()
    g = run_gpu(ctx, c["fixed"], c["moving"], c["fixed_range"], c["moving_range"], c["transforms"],
                c["bins"], c["q"])
    gmi, gov, gh = g
    assert np.array_equal(gh.reshape(len(gov), -1).sum(axis=1, dtype=np.int64), gov.astype(np.int64))
    assert np.all(np.isfinite(gmi)) and np.all(gmi[:, 0] >= -1e-12)
    pick = [0, 137, 555, 999]
    o = run_oracle(c["fixed"], c["moving"], c["fixed_range"], c["moving_range"], c["transforms"][pick],
                   c["bins"], c["q"])
    assert_parity((gmi[pick], gov[pick], gh[pick]), o, "full-size sample")


def test_timing_counts_launches(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.plain_translation(n=32)
    F = B.Volume.from_numpy(c["fixed"], 0, 255)
    tr = torch.from_numpy(c["transforms"]).cuda()
    ctx.timing(True)
    for _ in range(3):
        ctx.eval(F, F, tr, 32, [1.0])
    ctx.timing(False)
    ms, n = ctx.timing_read(B.TIMER_HARD)
    assert n == 3 and ms > 0
    ms, n = ctx.timing_read(B.TIMER_HARD)
    assert n == 0


def test_lds_atomic_probe(ctx):
    """The measurement probe returns a plausible peak: at least 1e12 and at
    most 256 CUs x 64 lanes x 2.4 GHz lane-atomics per second."""
    rate = ctx.probe_lds_atomics()
    assert 1e12 < rate < 256 * 64 * 2.4e9 * 1.01, rate


@pytest.mark.parametrize("bins,mrange", [(64, (0, 4095)), (256, (0, 255)), (200, (10, 3000))])
def test_maximum_edge_and_ragged_rows(ctx, bins, mrange):
    """Rows of 4096 voxels (the largest edge) with ragged y/z extents (3 and 2
    rows: partial 4-row groups), 16-bit and 8-bit oct volumes, u32 and packed
    LDS counters, under shifts and small rotations in the x-y plane."""
    rng = np.random.default_rng(13 + bins)
    fixed = inputs.random_volume(rng, (4096, 3, 2), np.uint16, 0, 4095)
    moving = inputs.random_volume(rng, (4096, 3, 3), np.uint16, mrange[0], mrange[1])
    mats = [T.translation((0, 0, 0)), T.translation((-37.25, 0.5, 0.25)), T.translation((4000.5, 1.0, 1.5))]
    for th in (0.02, -0.05):
        M = np.zeros((3, 4))
        M[:2, :2] = [[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]]
        M[2, 2] = 1.0
        M[:, 3] = (3.5, 1.0, 0.5)
        mats.append(M)
    mats = np.stack(mats).reshape(-1, 12)
    for flags in (0, 1):
        args = (fixed, moving, (0, 4095), mrange, mats, bins, [1.0, 1.5], flags)
        assert_parity(run_gpu(ctx, *args), run_oracle(*args), f"4096 rows bins={bins} flags={flags}")


def test_row_ranges_faces_turns_and_outside_rows(ctx):
    """Rows of 100 voxels (six 16-voxel steps and a ragged tail of 4): the
    sweep runs the steps where every lane of a 16 x 4 tile is inside the
    moving volume without per-voxel tests and, excluding the boundary,
    leaves out those where no lane can be.  Integer x-translations put the
    rows' ends exactly on the moving faces; quarter turns and mirrors about
    z give zero and negative x steps; scalings and large shifts put whole
    rows and tiles outside; large shears and a far translation take the
    path that tests every voxel."""
    rng = np.random.default_rng(17)
    fixed = inputs.random_volume(rng, (100, 23, 9), np.uint16, 0, 4095)
    moving = inputs.random_volume(rng, (90, 30, 11), np.uint16, 0, 4095)
    mats = [T.translation((tx, ty, tz)) for tx in (-16, -10, 0, 4, 10, 32, 89)
            for ty, tz in ((0, 0), (3.5, 1.0), (-2.0, -0.5))]
    quarter = [
        [[0, -1, 0, 29.0], [1, 0, 0, 0], [0, 0, 1, 0]],        # x steps along moving y
        [[-1, 0, 0, 89.0], [0, 1, 0, 0.5], [0, 0, 1, 1.0]],    # mirrored x
        [[0, 1, 0, 0], [-1, 0, 0, 99.0], [0, 0, 1, 0]],        # negative y steps
        [[0, 0, 1, 0], [0, 1, 0, 0], [1, 0, 0, 0]],            # x steps along moving z
        [[0, 0, 0, 40.0], [0, 1, 0, 0], [0, 0, 1, 0]],         # no x step at all
        [[1.1, 0.05, 0, -3.0], [-0.05, 1.1, 0, -1.0], [0, 0, 1.2, -0.5]],
        [[0.6, 0, 0, 20.25], [0, 0.9, 0, 2.0], [0, 0, 0.8, 1.0]],
        # entries too large for exact range arithmetic: every voxel tested
        [[1, 100.0, 0, -1150.5], [0, 1, 0, 2.0], [0, 0, 1, 0]],
        [[1, 0, 0, 200000.0], [0, 1, 0, 0], [0, 0, 1, 0]],
        [[1, 0, 0, 0], [0, 1, 0, 0], [0, -70.0, 1, 800.0]],
    ]
    mats = np.concatenate([np.stack(mats).reshape(-1, 12), np.asarray(quarter, dtype=np.float64).reshape(-1, 12)])
    for flags in (0, 1):
        args = (fixed, moving, (0, 4095), (0, 4095), mats, 64, [1.0, 0.5], flags)
        assert_parity(run_gpu(ctx, *args), run_oracle(*args), f"row ranges flags={flags}")
