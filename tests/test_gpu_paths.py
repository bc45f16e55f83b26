"""GPU parity of the parameter-space maps and their discrete gradient paths
(Results: translation, rotation and scale maps and the gradient paths on
them; Discussion: capture range).

* mi_map_paths through the C ABI against the oracle on the same seeded maps:
  successors, sinks and statistics bit-exact (integer results of the same
  fp64 comparisons), over ragged shapes, ties, plateaus, NaN points, both
  directions, off-centre centres, the maximum edge and a map larger than one
  pass of the grid-stride loop.
* maps.mi_map (batched mi_eval over a grid of one family) against the
  oracle's MI of the same matrices, within 1e-12 * max(1, |MI|), for every
  family and entropy, across several batches; a Mattes-style map (Parzen
  bins over a random subset of the voxels) within 1e-6.
"""
import zlib

import numpy as np
import pytest

import oracle
from oracle import paths as OP
from paper_1909_10690_amd import inputs, maps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1909_10690_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    c.close()


def seeded_map(shape, kind, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    if kind == "smooth":
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        v = (np.sin(x / 3.1) * np.cos(y / 2.3) + 0.5 * np.sin(z / 1.7 + x / 5.0)
             + 0.05 * rng.normal(size=shape))
    elif kind == "noise":
        v = rng.normal(size=shape)
    else:  # ties and plateaus, optionally with NaN points
        v = rng.integers(0, 4, size=shape).astype(np.float64)
        if kind == "nan":
            v[rng.random(shape) < 0.1] = np.nan
    return v


def gpu_paths(ctx, v, direction, centre):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    nxt, sink, stats = ctx.map_paths(t, direction, centre)
    torch.cuda.synchronize()
    return nxt.cpu().numpy().reshape(-1), sink.cpu().numpy().reshape(-1), tuple(stats.cpu().tolist())


CASES = [
    ((1, 1, 1), "noise"), ((1, 1, 9), "ties"), ((1, 6, 5), "nan"), ((3, 5, 7), "noise"),
    ((7, 5, 3), "ties"), ((11, 13, 17), "smooth"), ((9, 9, 9), "nan"), ((51, 51, 51), "smooth"),
    ((51, 51, 51), "ties"), ((2, 3, 4096), "noise"),
]


@pytest.mark.parametrize("shape,kind", CASES)
@pytest.mark.parametrize("direction", [1, -1])
def test_paths_match_oracle(ctx, shape, kind, direction):
    seed = zlib.crc32(repr((shape, kind, direction)).encode())
    v = seeded_map(shape, kind, seed)
    nz, ny, nx = shape
    for centre in ((nx // 2, ny // 2, nz // 2), (nx - 1, 0, nz - 1)):
        print(f"paths shape={shape} kind={kind} dir={direction} centre={centre}", flush=True)
        ref = OP.map_paths(v, direction, centre)
        nxt, sink, stats = gpu_paths(ctx, v, direction, centre)
        assert np.array_equal(nxt, ref["next"])
        assert np.array_equal(sink, ref["sink"])
        assert stats == tuple(ref["stats"])


def test_paths_beyond_one_grid_pass(ctx):
    """8.4 M points: more than the 8192 x 256 threads of one launch pass."""
    shape = (128, 256, 256)
    v = seeded_map(shape, "smooth", 11)
    ref = OP.map_paths(v, 1, (128, 128, 64))
    nxt, sink, stats = gpu_paths(ctx, v, 1, (128, 128, 64))
    assert np.array_equal(nxt, ref["next"]) and np.array_equal(sink, ref["sink"])
    assert stats == tuple(ref["stats"])


def test_paths_repeat_on_the_same_buffers(ctx):
    """Statistics start from zero on every call (no carry-over)."""
    import torch
    v = torch.from_numpy(seeded_map((9, 9, 9), "ties", 3)).cuda()
    a = [ctx.map_paths(v, 1)[2].cpu().tolist() for _ in range(3)]
    assert a[0] == a[1] == a[2]


@pytest.mark.parametrize("family", maps.FAMILIES)
def test_mi_map_matches_oracle(ctx, family):
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.same_image((20, 18, 16), seed=5, dtype=np.uint8)
    q = (1.0, 0.5, 2.0)
    n = 7
    ext = {"translation": 6.0, "rotation": 1.2, "scale": 0.3}[family]
    M = maps.map_transforms(family, n, (20, 18, 16), ext)
    fv = B.Volume.from_numpy(c["fixed"], *c["fixed_range"])
    mv = B.Volume.from_numpy(c["moving"], *c["moving_range"])
    print(f"mi_map family={family} n={n}", flush=True)
    got = maps.mi_map(ctx, fv, mv, family, n, ext, bins=c["bins"], q=q, batch=100).cpu().numpy()
    torch.cuda.synchronize()
    ref, _, _ = oracle.eval_hard(oracle.volume(c["fixed"], *c["fixed_range"]),
                                 oracle.volume(c["moving"], *c["moving_range"]), M, c["bins"], q)
    ref = ref.T.reshape(len(q), n, n, n)
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
    # same image on both sides: the identity at the centre is a local maximum
    # of the Shannon map
    nxt, _, _ = ctx.map_paths(torch.from_numpy(got[0]).cuda(), 1)
    ci = (3 * n + 3) * n + 3
    assert int(nxt.reshape(-1)[ci]) == ci


@pytest.mark.parametrize("family,ext", [("translation", 4.0), ("rotation", 1.0)])
def test_sampled_parzen_map_matches_oracle(ctx, family, ext):
    """A Mattes-style map (Parzen bins over a random 30% of the fixed voxels)
    against the oracle's sampled Parzen MI of the same matrices; rotation
    maps run in Z order and are put back in grid order."""
    from paper_1909_10690_amd import binding as B
    c = inputs.same_image((20, 18, 16), seed=6, dtype=np.uint8)
    q = (1.0, 2.0)
    n = 5
    M = maps.map_transforms(family, n, (20, 18, 16), ext)
    fv = B.Volume.from_numpy(c["fixed"], *c["fixed_range"])
    print(f"sampled Parzen map family={family}", flush=True)
    got = maps.mi_map(ctx, fv, fv, family, n, ext, bins=32, q=q,
                      flags=B.HIST_PARZEN | B.BOUNDARY_CLAMP, sample=(0.3, 44), batch=40).cpu().numpy()
    ref, _ = oracle.eval_parzen(oracle.volume(c["fixed"], *c["fixed_range"]),
                                oracle.volume(c["moving"], *c["moving_range"]), M, 32, q,
                                boundary=oracle.CLAMP, sample=(0.3, 44))
    ref = ref.T.reshape(len(q), n, n, n)
    assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref))
