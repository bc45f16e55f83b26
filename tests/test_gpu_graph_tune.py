"""GPU tests of HIP-graph replay (MI_USE_GRAPH) and of the autotuner.

Each graph is replayed several times with the program's own eager work and
synchronisations in between, and every replay is checked against an eager
call; the transforms are updated in place between replays, so a replay
must read the current device data.  The autotuner must leave results
bit-identical (the sweep is exact whatever its launch shape) and record its
choice in the cache file named by MI_TUNE_CACHE."""
import os

import numpy as np
import pytest

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


def _case():
    c = inputs.multimodal_sweep(shape_xyz=(96, 80, 48), n_tx=3, n_rot=3, n_scale=3)
    return c


def test_graph_replays_match_eager(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    c = _case()
    F = B.Volume.from_numpy(c["fixed"], 0, 4095)
    M = B.Volume.from_numpy(c["moving"], 0, 4095)
    base = torch.from_numpy(c["transforms"]).cuda()
    tr = base.clone()
    n, bins, q = len(base), c["bins"], c["q"]
    stream = torch.cuda.Stream()
    ws = torch.empty(ctx.workspace_size(F, M, n, bins, len(q)), dtype=torch.uint8, device="cuda")
    out = torch.empty((n, len(q)), dtype=torch.float64, device="cuda")
    hist = None
    rng = np.random.default_rng(0)
    for rep in range(4):
        if rep:
            # new transforms, written in place into the captured buffer
            shift = torch.from_numpy(rng.uniform(-2, 2, (n, 3))).cuda()
            tr.copy_(base)
            tr.view(n, 3, 4)[:, :, 3] += shift
        with torch.cuda.stream(stream):
            ctx.eval(F, M, tr, bins, q, flags=B.USE_GRAPH, out=out, workspace=ws, want_overlap=False)
        stream.synchronize()
        got = out.cpu().numpy().copy()
        ref, _, _ = ctx.eval(F, M, tr.clone(), bins, q)   # eager, default stream
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy()), f"replay {rep}"


def test_graph_gradient_and_pairs(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.parzen_gradient(n=40, n_transforms=5)
    F = B.Volume.from_numpy(c["fixed"], 0.0, 1.0)
    M = B.Volume.from_numpy(c["moving"], 0.0, 1.0)
    tr = torch.from_numpy(c["transforms"]).cuda()
    stream = torch.cuda.Stream()
    ws = torch.empty(ctx.workspace_size(F, M, 5, 32, 2, B.BOUNDARY_CLAMP | B.HIST_PARZEN | B.GRADIENT),
                     dtype=torch.uint8, device="cuda")
    ref_mi, ref_g = ctx.grad(F, M, tr, 32, [1.0, 1.5])
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(stream):
            mi, g = ctx.grad(F, M, tr, 32, [1.0, 1.5], flags=B.BOUNDARY_CLAMP | B.USE_GRAPH, workspace=ws)
        stream.synchronize()
        # fp64 atomics merge workgroup partials in any order
        np.testing.assert_allclose(mi.cpu().numpy(), ref_mi.cpu().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g.cpu().numpy(), ref_g.cpu().numpy(), rtol=1e-9, atol=1e-12)
        torch.cuda.synchronize()

    rng = np.random.default_rng(4)
    pairs = []
    for shape in [(20, 18, 16), (33, 9, 12), (17, 17, 40)]:
        f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
        m = inputs.random_volume(rng, shape, np.uint8, 0, 255)
        mats = inputs.random_affines(rng, 3, shape, rot=10, trans=3)
        pairs.append((B.Volume.from_numpy(f, 0, 255), B.Volume.from_numpy(m, 0, 255),
                      torch.from_numpy(mats).cuda()))
    ref = ctx.eval_pairs(pairs, 16, [1.0, 2.0]).cpu().numpy()
    for rep in range(3):
        with torch.cuda.stream(stream):
            got = ctx.eval_pairs(pairs, 16, [1.0, 2.0], flags=B.USE_GRAPH)
        stream.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref), f"pairs replay {rep}"


def test_tune_keeps_results_and_writes_cache(tmp_path):
    import torch
    from paper_1909_10690_amd import binding as B
    path = tmp_path / "tune.txt"
    os.environ["MI_TUNE_CACHE"] = str(path)
    try:
        ctx = B.Context(0)
        c = _case()
        F = B.Volume.from_numpy(c["fixed"], 0, 4095)
        M = B.Volume.from_numpy(c["moving"], 0, 4095)
        tr = torch.from_numpy(c["transforms"]).cuda()
        before, _, hb = ctx.eval(F, M, tr, 128, c["q"], want_hist=True)
        ctx.tune(F, M, tr, 128)
        after, _, ha = ctx.eval(F, M, tr, 128, c["q"], want_hist=True)
        torch.cuda.synchronize()
        assert torch.equal(hb, ha) and torch.equal(before, after)
        lines = [l for l in path.read_text().splitlines() if l.startswith("gemi-tune")]
        assert len(lines) == 1
        fields = lines[0].split()
        # key: 10 shape/bins/boundary/batch fields + oct8; then block, order, chunks, LDS layout
        assert fields[1:4] == ["96", "80", "48"] and fields[12] in ("256", "512", "1024")
        assert fields[15] in ("0", "1")
        ctx.close()
        ctx2 = B.Context(0)   # reads the cache file
        again, _, _ = ctx2.eval(F, M, tr, 128, c["q"])
        torch.cuda.synchronize()
        assert torch.equal(again, before)
        ctx2.close()
    finally:
        del os.environ["MI_TUNE_CACHE"]


def test_volume_preparation_reuse(ctx):
    """MI_VOLUMES_UNCHANGED reuses the workspace's prepared volumes: repeated
    calls match a fresh call, and a call whose volumes differ from the last
    preparation prepares again (the flag cannot make it wrong)."""
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.parzen_gradient(n=40, n_transforms=5)
    rng = np.random.default_rng(8)
    other = c["moving"][:, :, ::-1].copy()
    F = B.Volume.from_numpy(c["fixed"], 0.0, 1.0)
    M = B.Volume.from_numpy(c["moving"], 0.0, 1.0)
    M2 = B.Volume.from_numpy(other, 0.0, 1.0)
    tr = torch.from_numpy(c["transforms"]).cuda()
    ws = torch.empty(ctx.workspace_size(F, M, 5, 32, 2, B.BOUNDARY_CLAMP | B.HIST_PARZEN | B.GRADIENT),
                     dtype=torch.uint8, device="cuda")
    fl = B.BOUNDARY_CLAMP
    ref, ref_g = ctx.grad(F, M, tr, 32, [1.0, 1.5], flags=fl, workspace=ws)
    ref2, ref2_g = ctx.grad(F, M2, tr, 32, [1.0, 1.5], flags=fl, workspace=ws)
    for vol, r, rg in ((M, ref, ref_g), (M, ref, ref_g), (M2, ref2, ref2_g), (M2, ref2, ref2_g), (M, ref, ref_g)):
        mi, g = ctx.grad(F, vol, tr, 32, [1.0, 1.5], flags=fl | B.VOLUMES_UNCHANGED, workspace=ws)
        torch.cuda.synchronize()
        np.testing.assert_allclose(mi.cpu().numpy(), r.cpu().numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g.cpu().numpy(), rg.cpu().numpy(), rtol=1e-9, atol=1e-12)
    # hard path, same workspace: a different path prepares again
    h, _, _ = ctx.eval(B.Volume.from_numpy((c["fixed"] * 255).astype(np.uint8), 0, 255),
                       B.Volume.from_numpy((c["moving"] * 255).astype(np.uint8), 0, 255), tr, 32, [1.0],
                       flags=B.VOLUMES_UNCHANGED, workspace=torch.empty(1 << 26, dtype=torch.uint8, device="cuda"))
    h0, _, _ = ctx.eval(B.Volume.from_numpy((c["fixed"] * 255).astype(np.uint8), 0, 255),
                        B.Volume.from_numpy((c["moving"] * 255).astype(np.uint8), 0, 255), tr, 32, [1.0])
    torch.cuda.synchronize()
    assert torch.equal(h, h0)


def test_preparation_reuse_with_graphs(ctx):
    """Graphs always capture the preparation, and a graph launch updates the
    library's record of what the workspace holds, so interleaving graph
    replays and eager calls on two volume pairs with MI_VOLUMES_UNCHANGED
    stays correct."""
    import torch
    from paper_1909_10690_amd import binding as B
    c = inputs.parzen_gradient(n=40, n_transforms=5)
    F = B.Volume.from_numpy(c["fixed"], 0.0, 1.0)
    MA = B.Volume.from_numpy(c["moving"], 0.0, 1.0)
    MB = B.Volume.from_numpy(c["moving"][::-1].copy(), 0.0, 1.0)
    tr = torch.from_numpy(c["transforms"]).cuda()
    fl = B.BOUNDARY_CLAMP
    ws = torch.empty(ctx.workspace_size(F, MA, 5, 32, 2, fl | B.HIST_PARZEN | B.GRADIENT), dtype=torch.uint8,
                     device="cuda")
    refs = {}
    for name, M in (("A", MA), ("B", MB)):
        mi, _ = ctx.grad(F, M, tr, 32, [1.0, 1.5], flags=fl)
        torch.cuda.synchronize()
        refs[name] = mi.cpu().numpy()
    stream = torch.cuda.Stream()
    U, G = B.VOLUMES_UNCHANGED, B.USE_GRAPH
    outs = {n: (torch.empty((5, 2), dtype=torch.float64, device="cuda"),
                torch.empty((5, 2, 12), dtype=torch.float64, device="cuda")) for n in "AB"}

    def call(name, flags, graph):
        M = MA if name == "A" else MB
        if graph:
            with torch.cuda.stream(stream):
                mi, _ = ctx.grad(F, M, tr, 32, [1.0, 1.5], flags=flags | G, workspace=ws,
                                 out=outs[name])
            stream.synchronize()
        else:
            mi, _ = ctx.grad(F, M, tr, 32, [1.0, 1.5], flags=flags, workspace=ws)
            torch.cuda.synchronize()
        np.testing.assert_allclose(mi.cpu().numpy(), refs[name], rtol=1e-12, atol=1e-15)

    seq = [("A", fl, False), ("A", fl | U, True), ("B", fl, False), ("A", fl | U, True),
           ("B", fl | U, False), ("B", fl | U, True), ("A", fl | U, False), ("A", fl | U, True),
           ("B", fl | U, True), ("A", fl | U, False)]
    for name, flags, graph in seq:
        call(name, flags, graph)


def _pairs(seed, n=5, bins_dtype=np.uint8):
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(seed)
    pairs = []
    for k in range(n):
        shape = tuple(int(e) for e in rng.choice([24, 33, 40, 57], 3))
        f = inputs.random_volume(rng, shape, bins_dtype, 0, 255)
        m = inputs.random_volume(rng, shape, bins_dtype, 0, 255)
        mats = inputs.random_affines(rng, 3 + k % 3, shape, rot=10, trans=3)
        pairs.append((B.Volume.from_numpy(f, 0, 255), B.Volume.from_numpy(m, 0, 255),
                      torch.from_numpy(mats).cuda()))
    return pairs


@pytest.mark.parametrize("shape", ["256 65536 1 1", "1024 262144 0 0", "512 131072 0 1", "256 131072 1 0"])
def test_pairs_launch_shapes_keep_results(tmp_path, shape):
    """Every launch shape the pairs tuner can pick (workgroup size, slab
    voxels, 16-bit or u32 counters, work-item order), forced through the
    cache file, gives MI bit-identical to the default shape."""
    import torch
    from paper_1909_10690_amd import binding as B
    print(f"[tune] pairs shape {shape}", flush=True)
    path = tmp_path / "tune.txt"
    os.environ["MI_TUNE_CACHE"] = str(path)
    try:
        ctx = B.Context(0)
        pairs = _pairs(51)
        ref = ctx.eval_pairs(pairs, 64, [1.0, 2.0]).cpu().numpy()
        ctx.tune_pairs(pairs, 64)
        tuned = ctx.eval_pairs(pairs, 64, [1.0, 2.0]).cpu().numpy()
        assert np.array_equal(tuned, ref)
        lines = [l for l in path.read_text().splitlines() if l.startswith("gemi-tune-pairs")]
        assert len(lines) == 1
        f = lines[0].split()
        assert f[7] in ("256", "512", "1024") and f[9] in ("0", "1") and f[10] in ("0", "1")
        path.write_text(" ".join(f[:7] + shape.split()) + "\n")
        ctx.close()
        ctx2 = B.Context(0)  # reads the forced shape
        got = ctx2.eval_pairs(pairs, 64, [1.0, 2.0]).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, ref), shape
        ctx2.close()
    finally:
        del os.environ["MI_TUNE_CACHE"]


def test_pairs_preparation_reuse(ctx):
    """MI_VOLUMES_UNCHANGED on mi_eval_pairs keeps the pairs' fixed bins and
    oct volumes: repeated calls, transforms rewritten in place, graph
    replays and a different pair set through the same workspace (which
    prepares again) all match eager calls."""
    import torch
    from paper_1909_10690_amd import binding as B
    A, Bp = _pairs(61), _pairs(62, n=4)
    q = [1.0, 0.5]
    ws = torch.empty(max(ctx.pairs_workspace_size(A, 32, 2), ctx.pairs_workspace_size(Bp, 32, 2)),
                     dtype=torch.uint8, device="cuda")
    refA = ctx.eval_pairs(A, 32, q).cpu().numpy()
    refB = ctx.eval_pairs(Bp, 32, q).cpu().numpy()
    U = B.VOLUMES_UNCHANGED
    for k, (ps, ref) in enumerate([(A, refA), (A, refA), (Bp, refB), (Bp, refB), (A, refA)]):
        got = ctx.eval_pairs(ps, 32, q, flags=U, workspace=ws).cpu().numpy()
        assert np.array_equal(got, ref), k
    # transforms rewritten in place: the preparation stays, the matrices are read afresh
    rng = np.random.default_rng(63)
    for _, _, tr in A:
        tr.view(-1, 3, 4)[:, :, 3] += torch.from_numpy(rng.uniform(-1, 1, (tr.shape[0], 3))).cuda()
    fresh = ctx.eval_pairs(A, 32, q).cpu().numpy()
    got = ctx.eval_pairs(A, 32, q, flags=U, workspace=ws).cpu().numpy()
    assert np.array_equal(got, fresh) and not np.array_equal(fresh, refA)
    stream = torch.cuda.Stream()
    out = torch.empty_like(torch.from_numpy(fresh)).cuda()
    for rep in range(3):
        with torch.cuda.stream(stream):
            ctx.eval_pairs(A, 32, q, flags=U | B.USE_GRAPH, workspace=ws, out=out, stream=stream)
        stream.synchronize()
        assert np.array_equal(out.cpu().numpy(), fresh), f"replay {rep}"
        ctx.eval_pairs(Bp, 32, q, workspace=ws)  # eager work between replays: prepares B in the workspace
        torch.cuda.synchronize()


@pytest.mark.parametrize("forced", [None, "512 32 1024 128 -1", "1024 64 512 16 1", "256 96 256 64 0",
                                    "512 64 256 64 2"])
def test_parzen_tune_and_shapes_keep_results(tmp_path, forced):
    """mi_tune with MI_HIST_PARZEN picks forward and backward launch shapes;
    MI and gradients after tuning, and under shapes forced through the cache
    file (workgroup sizes, LDS band budgets, workgroup counts), match the
    default shape's: MI to the last bits (merge order of fp64 partial sums),
    gradients to the fp32 rounding of the per-lane partial sums, whose
    grouping follows the shape (1e-6 of the largest entry)."""
    import torch
    from paper_1909_10690_amd import binding as B
    print(f"[tune] parzen forced={forced}", flush=True)
    path = tmp_path / "tune.txt"
    os.environ["MI_TUNE_CACHE"] = str(path)
    try:
        ctx = B.Context(0)
        rng = np.random.default_rng(71)
        shape = (70, 52, 40)
        lab = inputs.render_labels(shape)
        f = inputs.intensities(lab, (0, 600, 1600, 2400), rng, 40.0, True, 0, 4095, np.uint16)
        m = inputs.intensities(lab, (0, 3600, 2000, 1200), rng, 40.0, True, 0, 4095, np.uint16)
        F, M = B.Volume.from_numpy(f, 0, 4095), B.Volume.from_numpy(m, 0, 4095)
        tr = torch.from_numpy(inputs.random_affines(rng, 3, shape, rot=6, trans=3)).cuda()
        q = [1.0, 1.3]
        fl = B.BOUNDARY_CLAMP
        ref_mi, ref_g = ctx.grad(F, M, tr, 256, q, flags=fl)
        ref_mi, ref_g = ref_mi.cpu().numpy(), ref_g.cpu().numpy()
        ctx.tune(F, M, tr, 256, flags=fl | B.HIST_PARZEN)
        lines = [l for l in path.read_text().splitlines() if l.startswith("gemi-tune-parzen")]
        assert len(lines) == 1
        fields = lines[0].split()
        assert fields[1:4] == ["70", "52", "40"] and fields[11] in ("256", "512", "1024") \
            and fields[13] in ("256", "512", "1024") and fields[15] in ("-1", "0", "1", "2")
        if forced:
            path.write_text(" ".join(fields[:11] + forced.split()) + "\n")
            ctx.close()
            ctx = B.Context(0)
        mi, g = ctx.grad(F, M, tr, 256, q, flags=fl)
        mi2, _, _ = ctx.eval(F, M, tr, 256, q, flags=fl | B.HIST_PARZEN)
        torch.cuda.synchronize()
        for a in (mi.cpu().numpy(), mi2.cpu().numpy()):
            np.testing.assert_allclose(a, ref_mi, rtol=1e-12, atol=1e-15)
        scale = np.abs(ref_g).max(axis=2, keepdims=True)
        assert (np.abs(g.cpu().numpy() - ref_g) <= 1e-6 * scale).all()
        ctx.close()
    finally:
        del os.environ["MI_TUNE_CACHE"]
