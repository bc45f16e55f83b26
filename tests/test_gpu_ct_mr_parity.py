"""Full-size parity of the Parzen gradient on the large cross-modality
workload: a 512x512x300 i16 CT-like fixed volume (1 mm) against a 256^3
u16 MR-like moving volume (2 mm), 256 Parzen bins, Shannon and Tsallis
q = 1.3 (the entropies of the Discussion's mixed strategy), clamp boundary
-- the per-iteration evaluation of gradient ascent on Eq. (3).

mi_grad and mi_eval (MI_HIST_PARZEN) through the C ABI against the CPU
oracle, element by element, on four transforms: the registration's start
(rot_z 6 deg, t (8, -5, 4) mm, scale 1.04), the truth (identity), a point
between them, and a tilt about x with a shear.  Bars as in the other Parzen
tests: MI within 1e-6 relative, gradient within 1e-4 |g_oracle|_inf per
transform and entropy, N exact.  At this size each workgroup lane sums
several hundred voxels' gradient terms and the 256-bin tables are split
into LDS bands over the ~125 occupied fixed-bin rows; the smaller Parzen
cases do not reach either."""
import numpy as np
import pytest

import oracle
from paper_1909_10690_amd import inputs
from paper_1909_10690_amd import transforms as T

pytestmark = pytest.mark.gpu

MI_TOL = 1e-6
GRAD_TOL = 1e-4
Q = [1.0, 1.3]


@pytest.fixture(scope="module")
def workload():
    print("[ct-mr parity] generating 512x512x300 i16 / 256^3 u16", flush=True)
    c = inputs.ct_mr_pair()
    nz, ny, nx = c["fixed"].shape
    centre = T.fixed_centre((nx, ny, nz), c["fixed_spacing"])
    st = c["start"]
    A0 = T.affine_matrix(st["angles"], st["scale"])
    params = [(A0, np.asarray(st["t"], dtype=np.float64)),
              (np.eye(3), np.zeros(3)),
              (T.affine_matrix((0.0, 0.0, 3.0), 1.02), np.asarray(st["t"]) / 2.0),
              (T.affine_matrix((2.5, -1.0, 0.0), (1.0, 0.98, 1.01), (0.02, 0.0, -0.01)), np.array([-3.0, 2.0, 1.5]))]
    # physical (mm) fixed -> moving matrices; the volumes carry their spacings and origins
    mats = np.stack([T.centred_matrix(A, t, centre).reshape(12) for A, t in params])
    F = oracle.volume(c["fixed"], *c["fixed_range"], c["fixed_spacing"], (0.0, 0.0, 0.0))
    M = oracle.volume(c["moving"], *c["moving_range"], c["moving_spacing"], c["moving_origin"])
    print("[ct-mr parity] oracle gradients of 4 transforms", flush=True)
    omi, og = oracle.parzen_grad(F, M, mats, 256, Q, oracle.CLAMP)
    return c, mats, omi, og


def test_ct_mr_full_size_gradient_parity(workload):
    import torch
    from paper_1909_10690_amd import binding as B
    c, mats, omi, og = workload
    print("[ct-mr parity] mi_grad / mi_eval on cuda:0", flush=True)
    ctx = B.Context(0)
    try:
        Fv = B.Volume.from_numpy(c["fixed"], *c["fixed_range"], spacing=c["fixed_spacing"])
        Mv = B.Volume.from_numpy(c["moving"], *c["moving_range"], spacing=c["moving_spacing"],
                                 origin=c["moving_origin"])
        tr = torch.from_numpy(mats).cuda()
        mi, g = ctx.grad(Fv, Mv, tr, 256, Q, flags=B.BOUNDARY_CLAMP)
        mi2, ov, _ = ctx.eval(Fv, Mv, tr, 256, Q, flags=B.BOUNDARY_CLAMP | B.HIST_PARZEN)
        # one transform per call, as the registration loop calls it
        single = [ctx.grad(Fv, Mv, tr[i:i + 1], 256, Q, flags=B.BOUNDARY_CLAMP) for i in range(len(mats))]
        torch.cuda.synchronize()
    finally:
        ctx.close()
    gmi, gg, gmi2 = mi.cpu().numpy(), g.cpu().numpy(), mi2.cpu().numpy()
    assert np.array_equal(ov.cpu().numpy(), np.full(len(mats), c["fixed"].size)), "clamp: every voxel counts"
    for label, a in (("mi_grad", gmi), ("mi_eval", gmi2)):
        err = np.abs(a - omi) / np.maximum(1.0, np.abs(omi))
        assert err.max() <= MI_TOL, f"{label} MI rel err {err.max()}"
    scale = np.abs(og).max(axis=2)
    for label, gr in [("batch", gg)] + [(f"single {i}", s[1].cpu().numpy()) for i, s in enumerate(single)]:
        if label.startswith("single"):
            i = int(label.split()[1])
            diff = np.abs(gr[0] - og[i]).max(axis=1)
            assert (diff <= GRAD_TOL * scale[i]).all(), f"{label}: gradient err {diff} scale {scale[i]}"
        else:
            diff = np.abs(gr - og).max(axis=2)
            assert (diff <= GRAD_TOL * scale).all(), f"{label}: gradient err {diff / scale}"
