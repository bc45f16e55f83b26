"""Batches whose grid would pass the dispatch's 32-bit work-item count are
split by the library into launches of whole transforms (below 2^31
work-items each); every transform of the batch is evaluated.  Both cases
below give more than 2^32 work-items in one grid (1.1 M transforms x at
least 8 workgroups x 512 or 1024 threads), which wrapped before the split
and left the tail of the batch unevaluated.

* mi_eval (hard bins) of 1.1 M fractional translations on a 16^3 volume:
  a sample of rows, the last ones included (the transforms a wrapped grid
  would drop), against the oracle within 1e-12 * max(1, |MI|), and the
  overlap counts exactly.
* mi_grad (Parzen) of 1.1 M transforms: sampled rows, the tail included,
  equal to the same transforms in a small batch (to 1e-9: the fp64 merges
  of partial tables run in scheduling order).
"""
import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1909_10690_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    c.close()


def translations(rng, n, reach):
    M = np.zeros((n, 3, 4))
    M[:, 0, 0] = M[:, 1, 1] = M[:, 2, 2] = 1.0
    M[:, :, 3] = rng.uniform(-reach, reach, (n, 3))
    return M.reshape(n, 12)


def sample_rows(n):
    return np.unique(np.concatenate([np.arange(0, n, n // 25), np.arange(n - 20, n)]))


def test_hard_batch_beyond_one_dispatch(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(51)
    shape = (16, 16, 16)
    f = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    m = inputs.random_volume(rng, shape, np.uint8, 0, 255)
    n = 1_100_000
    M = translations(rng, n, 3.0)
    F, Mv = B.Volume.from_numpy(f, 0, 255), B.Volume.from_numpy(m, 0, 255)
    q = (1.0, 2.0)
    print(f"hard batch n={n}", flush=True)
    mi, ov, _ = ctx.eval(F, Mv, torch.from_numpy(M).cuda(), 8, q)
    torch.cuda.synchronize()
    mi, ov = mi.cpu().numpy(), ov.cpu().numpy()
    rows = sample_rows(n)
    ref, ref_ov, _ = oracle.eval_hard(oracle.volume(f, 0, 255), oracle.volume(m, 0, 255), M[rows], 8, q)
    assert np.array_equal(ov[rows], ref_ov)
    assert np.all(np.abs(mi[rows] - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))


def test_parzen_grad_batch_beyond_one_dispatch(ctx):
    import torch
    from paper_1909_10690_amd import binding as B
    rng = np.random.default_rng(52)
    shape = (16, 16, 16)
    f = inputs.random_volume(rng, shape, np.float32, 0.0, 1.0)
    m = inputs.random_volume(rng, shape, np.float32, 0.0, 1.0)
    n = 1_100_000
    M = translations(rng, n, 2.0)
    F, Mv = B.Volume.from_numpy(f, 0.0, 1.0), B.Volume.from_numpy(m, 0.0, 1.0)
    q = (1.0, 1.5)
    print(f"parzen grad batch n={n}", flush=True)
    mi, g = ctx.grad(F, Mv, torch.from_numpy(M).cuda(), 8, q)
    torch.cuda.synchronize()
    rows = sample_rows(n)
    mi_s, g_s = ctx.grad(F, Mv, torch.from_numpy(M[rows]).cuda(), 8, q)
    torch.cuda.synchronize()
    mi, g = mi.cpu().numpy()[rows], g.cpu().numpy()[rows]
    mi_s, g_s = mi_s.cpu().numpy(), g_s.cpu().numpy()
    assert np.all(np.isfinite(mi)) and np.all(np.isfinite(g))
    assert np.all(np.abs(mi - mi_s) <= 1e-9 * np.maximum(1.0, np.abs(mi_s)))
    assert np.all(np.abs(g - g_s) <= 1e-9 * np.maximum(1.0, np.abs(g_s).max()))
