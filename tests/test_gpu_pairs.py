"""GPU parity of the persistent multi-pair path (mi_eval_pairs through the
C ABI) against the CPU oracle: every pair's MI within 1e-12 * max(1, |MI|)
(histograms are exact, so any miscounted voxel would show), for pairs of
uneven sizes, dtypes and transform counts in one launch."""
import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1909_10690_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    c.close()


def run_pairs(ctx, pairs, bins, q, flags):
    import torch
    from paper_1909_10690_amd import binding as B
    gp = [(B.Volume.from_numpy(p["fixed"], *p["frange"]), B.Volume.from_numpy(p["moving"], *p["mrange"]),
           torch.from_numpy(np.ascontiguousarray(p["transforms"].reshape(-1, 12))).cuda()) for p in pairs]
    mi = ctx.eval_pairs(gp, bins, q, flags=flags)
    torch.cuda.synchronize()
    return mi.cpu().numpy()


def oracle_pairs(pairs, bins, q, flags):
    out = []
    for p in pairs:
        mi, _, _ = oracle.eval_hard(oracle.volume(p["fixed"], *p["frange"]),
                                    oracle.volume(p["moving"], *p["mrange"]), p["transforms"], bins, q,
                                    boundary=flags & 1,
                                    form=oracle.PSEUDOADDITIVE if flags & 0x10 else oracle.ADDITIVE)
        out.append(mi)
    return np.concatenate(out) if out else np.zeros((0, len(q)))


def check(g, o):
    nan = np.isnan(o)
    assert np.array_equal(np.isnan(g), nan)
    err = np.abs(g[~nan] - o[~nan]) / np.maximum(1.0, np.abs(o[~nan]))
    assert err.size == 0 or err.max() <= 1e-12, err.max()


def mixed_pairs(seed, n=7):
    rng = np.random.default_rng(seed)
    kinds = [(np.uint8, (0, 255)), (np.uint16, (0, 4095)), (np.int16, (-1000, 1500))]
    pairs = []
    for i in range(n):
        shape = tuple(int(e) for e in rng.choice([9, 17, 24, 33, 40, 67], 3))
        dt, r = kinds[i % 3]
        lab = inputs.render_labels(shape)
        lev = np.linspace(r[0] + 10, r[1] - 10, 4)
        f = inputs.intensities(lab, lev, rng, 10.0, False, r[0], r[1], dt)
        truth = T.centred_matrix(T.affine_matrix(rng.uniform(-5, 5, 3)), rng.uniform(-2, 2, 3), T.fixed_centre(shape))
        m = inputs.intensities(inputs.render_labels(shape, inv_map=inputs.invert(truth)), lev[::-1], rng, 10.0,
                               False, r[0], r[1], dt)
        nt = int(rng.integers(0, 6))
        mats = list(inputs.random_affines(rng, nt, shape, rot=20, trans=5).reshape(-1, 3, 4))
        if i == 2:
            mats += [T.translation((np.nan, 0, 0)), T.translation((500, 0, 0))]
        mats = np.stack(mats).reshape(-1, 12) if mats else np.zeros((0, 12))
        pairs.append(dict(fixed=f, moving=m, frange=r, mrange=r, transforms=mats))
    return pairs


@pytest.mark.parametrize("bins,flags", [(32, 0), (64, 1), (200, 0), (7, 0x10)])
def test_mixed_pairs(ctx, bins, flags):
    pairs = mixed_pairs(bins + flags)
    q = [1.0, 0.5, 2.0]
    check(run_pairs(ctx, pairs, bins, q, flags), oracle_pairs(pairs, bins, q, flags))


def test_runs_of_pairs_without_transforms(ctx):
    """Pairs with no transforms have no work items: a workgroup's queue moves
    past runs of them (the first pair, three in a row, the last) to the next
    pair that has items."""
    rng = np.random.default_rng(41)
    pairs = []
    for i in range(8):
        shape = tuple(int(e) for e in rng.choice([12, 17, 24], 3))
        f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
        m = inputs.random_volume(rng, shape, np.uint8, 0, 255)
        nt = 0 if i in (0, 2, 3, 4, 7) else 3
        mats = inputs.random_affines(rng, nt, shape, rot=10, trans=3)
        pairs.append(dict(fixed=f, moving=m, frange=(0, 255), mrange=(0, 255), transforms=mats))
    q = [1.0, 2.0]
    got = run_pairs(ctx, pairs, 32, q, 0)
    assert got.shape == (9, 2)
    check(got, oracle_pairs(pairs, 32, q, 0))


def test_pairs_equal_single_pair_calls(ctx):
    """One persistent launch over many pairs gives exactly what mi_eval gives
    pair by pair."""
    import torch
    from paper_1909_10690_amd import binding as B
    pairs = mixed_pairs(5, n=9)
    q = [1.0, 1.5]
    got = run_pairs(ctx, pairs, 64, q, 0)
    rows = []
    for p in pairs:
        if len(p["transforms"]) == 0:
            continue
        F = B.Volume.from_numpy(p["fixed"], *p["frange"])
        M = B.Volume.from_numpy(p["moving"], *p["mrange"])
        mi, _, _ = ctx.eval(F, M, torch.from_numpy(p["transforms"]).cuda(), 64, q)
        rows.append(mi.cpu().numpy())
    ref = np.concatenate(rows)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[~np.isnan(got)], ref[~np.isnan(ref)])


def test_uneven_pairs_full_size_sampled(ctx):
    """The 256-pair, 16-rigid-transforms-each, 64-bin launch; sampled pairs
    against the oracle."""
    raw = inputs.uneven_pairs()
    pairs = [dict(fixed=p["fixed"], moving=p["moving"], frange=(0, 255), mrange=(0, 255),
                  transforms=p["transforms"]) for p in raw]
    g = run_pairs(ctx, pairs, 64, [1.0], 0)
    assert g.shape == (256 * 16, 1) and np.all(np.isfinite(g)) and np.all(g >= -1e-12)
    for k in (0, 97, 255):
        o = oracle_pairs([pairs[k]], 64, [1.0], 0)
        check(g[16 * k:16 * (k + 1)], o)


def test_u8_pairs_vector_and_scalar_prep(ctx):
    """All-u8 pairs (8-bit oct volumes for every pair) through every branch
    of the preparation: moving rows of even length take the two-voxels-per-
    lane path, odd lengths the per-voxel path, with ragged plane runs and
    slice blocks (depths not a multiple of 8); fixed volumes take 16-byte
    accesses except in a ragged last chunk.  Volumes that start 1, 4 or 8
    bytes into their device buffers (1: odd addresses, per-voxel moving path;
    4 and 8: not 16-byte aligned, per-voxel fixed path) give the same
    result."""
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(31)
    pairs = []
    for shape in [(20, 9, 16), (13, 12, 24), (40, 17, 12), (36, 24, 5), (17, 9, 8), (11, 7, 9)]:
        f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
        m = inputs.random_volume(rng, shape, np.uint8, 20, 230)
        mats = inputs.random_affines(rng, 3, shape, rot=15, trans=4)
        pairs.append(dict(fixed=f, moving=m, frange=(0, 255), mrange=(20, 230), transforms=mats))
    q = [1.0, 1.5]
    check(run_pairs(ctx, pairs, 48, q, 0), oracle_pairs(pairs, 48, q, 0))
    # the first pair again, its volumes `shift` bytes into their device buffers
    p = pairs[0]
    ref = oracle_pairs([p], 48, q, 0)
    nz, ny, nx = p["fixed"].shape
    for shift in (1, 4, 8):
        print(f"prep shift={shift}", flush=True)
        fb = torch.empty(p["fixed"].size + shift, dtype=torch.uint8, device="cuda")
        mb = torch.empty(p["moving"].size + shift, dtype=torch.uint8, device="cuda")
        fb[shift:].copy_(torch.from_numpy(p["fixed"].reshape(-1)))
        mb[shift:].copy_(torch.from_numpy(p["moving"].reshape(-1)))
        F = B.Volume(fb[shift:].view(nz, ny, nx), 0, 255)
        M = B.Volume(mb[shift:].view(nz, ny, nx), 20, 230)
        got = ctx.eval_pairs([(F, M, torch.from_numpy(p["transforms"]).cuda())], 48, q).cpu().numpy()
        check(got, ref)
