"""GPU parity of random subsampling (mi_eval_sampled through the C ABI)
against the CPU oracle (Discussion: Mattes' MI samples voxels at random).

Hard histograms over the kept voxels are bit-exact and MI within
1e-12 * max(1, |MI|); Parzen MI within 1e-6 relative with the normaliser
exact.  Cases: ragged shapes and dtypes, both boundary modes, the packed
16-bit LDS layout with more than 65535 samples per workgroup (counted in
flushed spans), fraction 1 against mi_eval, tiny fractions (possibly no
sample at all), seeds, graph replays, and the benchmark-sized volume.
"""
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


def gpu_sampled(ctx, f, m, frange, mrange, mats, bins, q, fraction, seed, flags=0, want_hist=True):
    import torch
    from paper_1909_10690_amd import binding as B
    F = B.Volume.from_numpy(f, *frange)
    M = B.Volume.from_numpy(m, *mrange)
    tr = torch.from_numpy(np.ascontiguousarray(np.asarray(mats, dtype=np.float64).reshape(-1, 12))).cuda()
    mi, ov, h = ctx.eval_sampled(F, M, tr, bins, q, fraction=fraction, seed=seed, flags=flags,
                                 want_hist=want_hist)
    torch.cuda.synchronize()
    return mi.cpu().numpy(), ov.cpu().numpy(), None if h is None else h.cpu().numpy().astype(np.uint32)


def close(a, b, tol=1e-12):
    return np.all(np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b)))


CASES = [
    # shape (x, y, z), fixed dtype/range, moving dtype/range, bins, fraction, seed, clamp
    ((17, 13, 9), np.uint8, (0, 255), np.uint8, (0, 255), 32, 0.3, 1, False),
    ((33, 20, 11), np.uint16, (0, 4095), np.uint16, (0, 4095), 128, 0.1, 2 ** 63 + 11, False),
    ((24, 24, 24), np.int16, (-1000, 1500), np.uint16, (0, 4095), 256, 0.5, 7, True),
    ((2, 2, 2), np.uint8, (0, 255), np.uint8, (0, 255), 2, 0.9, 3, False),
    ((40, 3, 2), np.uint8, (0, 255), np.uint16, (0, 65535), 64, 0.25, 0, True),
]


@pytest.mark.parametrize("shape,fdt,fr,mdt,mr,bins,fraction,seed,clamp", CASES)
def test_hard_sampled_matches_oracle(ctx, shape, fdt, fr, mdt, mr, bins, fraction, seed, clamp):
    rng = np.random.default_rng(abs(hash(shape)) % 1000)
    f = inputs.random_volume(rng, shape, fdt, *fr)
    m = inputs.random_volume(rng, shape, mdt, *mr)
    mats = np.concatenate([inputs.random_affines(rng, 6, shape, rot=20, trans=3),
                           T.translation((0.5, -1.0, 0.25)).reshape(1, 12)])
    q = (1.0, 0.5, 2.0)
    print(f"hard sampled shape={shape} bins={bins} fraction={fraction} seed={seed}", flush=True)
    mi, ov, h = gpu_sampled(ctx, f, m, fr, mr, mats, bins, q, fraction, seed, flags=int(clamp))
    rmi, rov, rh = oracle.eval_hard(oracle.volume(f, *fr), oracle.volume(m, *mr), mats, bins, q,
                                    boundary=int(clamp), want_hist=True, sample=(fraction, seed))
    assert np.array_equal(h, rh)
    assert np.array_equal(ov, rov)
    assert close(mi, rmi)


def test_packed_counters_beyond_one_span(ctx):
    """More than 65535 samples per workgroup with 16-bit counters: the spans
    are flushed in turn.  Fraction 1 equals mi_eval bit for bit; a sampled
    run matches the oracle on a few transforms."""
    import torch
    from paper_1909_10690_amd import binding as B
    shape = (128, 128, 128)
    rng = np.random.default_rng(5)
    f = inputs.random_volume(rng, shape, np.uint16, 0, 4095)
    m = inputs.random_volume(rng, shape, np.uint16, 0, 4095)
    mats = inputs.random_affines(rng, 256, shape, rot=5, trans=2)
    F, Mv = B.Volume.from_numpy(f, 0, 4095), B.Volume.from_numpy(m, 0, 4095)
    tr = torch.from_numpy(mats).cuda()
    print("packed spans: fraction 1 vs mi_eval, 256 transforms of 128^3", flush=True)
    _, ov_a, h_a = ctx.eval_sampled(F, Mv, tr, 256, (1.0,), fraction=1.0, seed=9, want_hist=True)
    _, ov_b, h_b = ctx.eval(F, Mv, tr, 256, (1.0,), want_hist=True)
    torch.cuda.synchronize()
    assert torch.equal(h_a, h_b) and torch.equal(ov_a, ov_b)
    mi, ov, h = ctx.eval_sampled(F, Mv, tr, 256, (1.0, 1.5), fraction=0.6, seed=21, want_hist=True)
    torch.cuda.synchronize()
    pick = [0, 77, 255]
    rmi, rov, rh = oracle.eval_hard(oracle.volume(f, 0, 4095), oracle.volume(m, 0, 4095), mats[pick], 256,
                                    (1.0, 1.5), want_hist=True, sample=(0.6, 21))
    assert np.array_equal(h.cpu().numpy()[pick].astype(np.uint32), rh)
    assert np.array_equal(ov.cpu().numpy()[pick], rov)
    assert close(mi.cpu().numpy()[pick], rmi)


def test_tiny_fraction_and_seeds(ctx):
    rng = np.random.default_rng(8)
    shape = (10, 9, 8)
    f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    mats = inputs.random_affines(rng, 3, shape)
    # about 0.0007 expected samples: almost surely none -> MI 0, overlap 0
    mi, ov, h = gpu_sampled(ctx, f, f, (0, 255), (0, 255), mats, 16, (1.0,), 1e-6, 4)
    rmi, rov, _ = oracle.eval_hard(oracle.volume(f, 0, 255), oracle.volume(f, 0, 255), mats, 16, (1.0,),
                                   sample=(1e-6, 4))
    assert np.array_equal(ov, rov) and close(mi, rmi)
    a = gpu_sampled(ctx, f, f, (0, 255), (0, 255), mats, 16, (1.0,), 0.5, 4)
    b = gpu_sampled(ctx, f, f, (0, 255), (0, 255), mats, 16, (1.0,), 0.5, 4)
    c = gpu_sampled(ctx, f, f, (0, 255), (0, 255), mats, 16, (1.0,), 0.5, 5)
    assert np.array_equal(a[2], b[2]) and not np.array_equal(a[2], c[2])


@pytest.mark.parametrize("moving_float,clamp", [(True, True), (False, True), (True, False)])
def test_parzen_sampled_matches_oracle(ctx, moving_float, clamp):
    from paper_1909_10690_amd import binding as B
    c = inputs.parzen_gradient(n=40, seed=3, n_transforms=6)
    f, m = c["fixed"], c["moving"]
    if not moving_float:
        m = np.rint(m * 4095).astype(np.uint16)
    mr = (0.0, 1.0) if moving_float else (0, 4095)
    q = (1.0, 1.5)
    flags = B.HIST_PARZEN | (B.BOUNDARY_CLAMP if clamp else 0)
    print(f"parzen sampled float={moving_float} clamp={clamp}", flush=True)
    mi, ov, _ = gpu_sampled(ctx, f, m, (0.0, 1.0), mr, c["transforms"], 64, q, 0.3, 17, flags=flags,
                            want_hist=False)
    rmi, rov = oracle.eval_parzen(oracle.volume(f, 0.0, 1.0), oracle.volume(m, *mr), c["transforms"], 64, q,
                                  boundary=int(clamp), sample=(0.3, 17))
    assert np.array_equal(ov, rov)
    assert np.all(np.abs(mi - rmi) <= 1e-6 * np.abs(rmi))


def test_parzen_fraction_one_equals_mi_eval(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.parzen_gradient(n=48, seed=4, n_transforms=5)
    F = B.Volume.from_numpy(c["fixed"], 0.0, 1.0)
    Mv = B.Volume.from_numpy(c["moving"], 0.0, 1.0)
    tr = torch.from_numpy(c["transforms"]).cuda()
    a, oa, _ = ctx.eval_sampled(F, Mv, tr, 256, (1.0, 0.7), fraction=1.0, seed=1, flags=B.HIST_PARZEN)
    b, ob, _ = ctx.eval(F, Mv, tr, 256, (1.0, 0.7), flags=B.HIST_PARZEN)
    torch.cuda.synchronize()
    assert torch.equal(oa, ob)
    assert close(a.cpu().numpy(), b.cpu().numpy())


def test_sampled_graph_replays(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(12)
    shape = (30, 20, 10)
    f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    F = B.Volume.from_numpy(f, 0, 255)
    tr = torch.from_numpy(inputs.random_affines(rng, 8, shape)).cuda()
    s = torch.cuda.Stream()
    ws = torch.empty(ctx.workspace_size(F, F, 8, 32, 1, B.SAMPLED), dtype=torch.uint8, device="cuda")
    eager, _, _ = ctx.eval_sampled(F, F, tr, 32, (1.0,), fraction=0.4, seed=3, workspace=ws)
    torch.cuda.synchronize()
    out = torch.empty_like(eager)
    for _ in range(3):
        with torch.cuda.stream(s):
            ctx.eval_sampled(F, F, tr, 32, (1.0,), fraction=0.4, seed=3, flags=B.USE_GRAPH, out=out,
                             want_overlap=False, workspace=ws, stream=s)
        s.synchronize()
        assert torch.equal(out, eager)
        out.zero_()
        torch.cuda.synchronize()
