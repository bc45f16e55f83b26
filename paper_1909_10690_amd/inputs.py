"""Seeded synthetic inputs: head phantoms, volume pairs and transform batches.

The paper measures on HCP Young Adult 3T structural brain images
(Methodology), which are not available here; these phantoms stand in for
them.  Each workload mirrors one measured configuration: a plain 64^3 u8
translation sweep, a 256x256x180 u16 multi-modal sweep of 1000 transforms,
a 128^3 f32 Parzen/gradient case, 256 uneven u8 pairs, and a large CT/MR
pair.  A phantom is a set of nested ellipsoids (background, CSF, grey,
white matter) with two ventricles and one off-centre lesion that breaks
mirror symmetry; intensities per class plus Gaussian or Rician noise.

This module holds no part of the metric's arithmetic.  Moving volumes are
rendered analytically at the inverse-transformed position of each moving
voxel (no interpolation), except the plain translation workload, whose
moving volume is the fixed one resampled by scipy's order-1 spline
(trilinear, edge-clamped).  Transforms are physical fixed -> moving
matrices; every workload but the CT/MR pair has unit spacings and zero
origins, where physical and voxel coordinates coincide.
"""
from __future__ import annotations

import numpy as np

from . import transforms as T

BG, CSF, GREY, WHITE, CALC = 0, 1, 2, 3, 4


def _ellipsoid(p, c, a):
    return (((p[0] - c[0]) / a[0]) ** 2 + ((p[1] - c[1]) / a[1]) ** 2 +
            ((p[2] - c[2]) / a[2]) ** 2) <= 1.0


# Off-axis calcification-like spheres (label CALC; centre and radius in
# units of the head's half-extent) for workloads registered with a full
# affine: nested, axis-aligned ellipsoids alone are mapped onto their
# rotated copies by a symmetric linear map, so a rotation could be traded
# for a shear.
FEATURES = ((-0.35, 0.30, -0.25, 0.09), (0.40, -0.20, 0.10, 0.08), (-0.20, -0.40, 0.30, 0.10),
            (0.15, 0.45, -0.35, 0.07), (-0.45, -0.05, 0.05, 0.08), (0.30, 0.10, 0.45, 0.09))


def head_labels(points_xyz, shape_xyz, jitter: float = 1.0, lesion: bool = True,
                scale_xyz=(1.0, 1.0, 1.0), features: bool = False) -> np.ndarray:
    """Tissue labels at points given in index units of a volume of
    ``shape_xyz``; ``points_xyz`` is a sequence of three broadcastable
    coordinate arrays (x, y, z); ``scale_xyz`` stretches the anatomy per axis;
    ``features`` adds the FEATURES spheres."""
    n = np.asarray(shape_xyz, dtype=np.float64)
    c = (n - 1.0) / 2.0
    h = n / 2.0 * np.asarray(scale_xyz, dtype=np.float64) * jitter
    shape = np.broadcast_shapes(*(np.shape(v) for v in points_xyz))
    lab = np.zeros(shape, dtype=np.uint8)
    lab[_ellipsoid(points_xyz, c, h * np.array([0.85, 0.75, 0.80]))] = CSF
    lab[_ellipsoid(points_xyz, c, h * np.array([0.78, 0.68, 0.72]))] = GREY
    lab[_ellipsoid(points_xyz, c, h * np.array([0.60, 0.50, 0.55]))] = WHITE
    vent = h * np.array([0.12, 0.20, 0.15])
    for sx in (-1.0, 1.0):
        lab[_ellipsoid(points_xyz, c + np.array([sx * 0.12 * h[0], 0.0, 0.0]), vent)] = CSF
    if lesion:
        lc = c + h * np.array([0.30, 0.25, 0.20])
        lab[_ellipsoid(points_xyz, lc, h * 0.08)] = CSF
    if features:
        for fx, fy, fz, r in FEATURES:
            lab[_ellipsoid(points_xyz, c + h * np.array([fx, fy, fz]), h * r)] = CALC
    return lab


def _slab_points(shape_xyz, z0: int, z1: int, M=None):
    """Coordinates (x, y, z) of voxels [z0, z1) x all y x all x, mapped by
    the 3x4 matrix M if given; separable, so built by broadcasting 1-D axes."""
    nx, ny, _ = shape_xyz
    x = np.arange(nx, dtype=np.float32)[None, None, :]
    y = np.arange(ny, dtype=np.float32)[None, :, None]
    z = np.arange(z0, z1, dtype=np.float32)[:, None, None]
    if M is None:
        return x, y, z
    M = np.asarray(M, dtype=np.float32)
    return tuple(M[r, 0] * x + M[r, 1] * y + M[r, 2] * z + M[r, 3] for r in range(3))


def render_labels(shape_xyz, inv_map=None, jitter=1.0, lesion=True, scale_xyz=(1.0, 1.0, 1.0),
                  anatomy_shape_xyz=None, chunk=64, features=False) -> np.ndarray:
    """Label volume [nz][ny][nx].  ``inv_map`` (3x4) takes this volume's voxel
    index to the anatomy's index frame (``anatomy_shape_xyz``, default the
    same shape); identity when None."""
    nx, ny, nz = shape_xyz
    ana = shape_xyz if anatomy_shape_xyz is None else anatomy_shape_xyz
    out = np.empty((nz, ny, nx), dtype=np.uint8)
    for z0 in range(0, nz, chunk):
        z1 = min(nz, z0 + chunk)
        p = _slab_points(shape_xyz, z0, z1, inv_map)
        out[z0:z1] = np.broadcast_to(head_labels(p, ana, jitter, lesion, scale_xyz, features),
                                     (z1 - z0, ny, nx))
    return out


def invert(M: np.ndarray) -> np.ndarray:
    A = np.linalg.inv(M[:, :3])
    Mi = np.zeros((3, 4))
    Mi[:, :3] = A
    Mi[:, 3] = -A @ M[:, 3]
    return Mi


def intensities(labels: np.ndarray, levels, rng: np.random.Generator, sigma: float, rician: bool,
                lo: float, hi: float, dtype) -> np.ndarray:
    """Class intensities + N(0, sigma) (or Rician magnitude) noise, rounded and clipped."""
    s = np.asarray(levels, dtype=np.float32)[labels]
    if rician:
        n1 = rng.standard_normal(labels.shape, dtype=np.float32)
        n2 = rng.standard_normal(labels.shape, dtype=np.float32)
        v = np.sqrt((s + np.float32(sigma) * n1) ** 2 + (np.float32(sigma) * n2) ** 2)
    else:
        v = s + np.float32(sigma) * rng.standard_normal(labels.shape, dtype=np.float32)
    v = np.clip(np.rint(v), lo, hi)
    return v.astype(dtype)


def resample_trilinear(vol: np.ndarray, M: np.ndarray) -> np.ndarray:
    """out[i] = vol(M^-1 i) by scipy's order-1 spline, edge values clamped."""
    from scipy import ndimage
    nz, ny, nx = vol.shape
    Mi = invert(M)
    p = [np.broadcast_to(v, (nz, ny, nx)).astype(np.float64) for v in _slab_points((nx, ny, nz), 0, nz, Mi)]
    coords = np.stack([p[2], p[1], p[0]])
    return ndimage.map_coordinates(vol.astype(np.float64), coords, order=1, mode="nearest")


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def plain_translation(n: int = 64, seed: int = 0) -> dict:
    """64^3 u8 head phantom; moving = fixed translated by (3.5, -2, 1.25)
    voxels (trilinear); 32 bins; Shannon over 21 x-translations in [-10, 10]."""
    rng = np.random.default_rng(seed)
    lab = render_labels((n, n, n))
    fixed = intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.uint8)
    truth = T.translation((3.5, -2.0, 1.25))
    moving = np.clip(np.rint(resample_trilinear(fixed, truth)), 0, 255).astype(np.uint8)
    mats = np.stack([T.translation((tx, -2.0, 1.25)) for tx in np.arange(-10, 11, dtype=np.float64)])
    return dict(name="plain-translation 64^3 u8", fixed=fixed, moving=moving, fixed_range=(0, 255),
                moving_range=(0, 255), transforms=mats.reshape(-1, 12), bins=32, q=[1.0], truth=truth)


def multimodal_sweep(shape_xyz=(256, 256, 180), seed: int = 1, n_tx=10, n_rot=10, n_scale=10) -> dict:
    """256x256x180 u16 T1-like fixed vs T2-like moving (non-monotone remap)
    under rot_z 5 deg, t (4,-3,2), scale 1.03; 128 bins; Shannon and Tsallis
    q in {0.5, 0.8, 1.2, 1.5, 2.0}; grid of tx x rot_z x scale transforms."""
    rng = np.random.default_rng(seed)
    lab_f = render_labels(shape_xyz)
    fixed = intensities(lab_f, (0, 600, 1600, 2400), rng, 40.0, True, 0, 4095, np.uint16)
    truth = T.centred_matrix(T.affine_matrix((0, 0, 5.0), 1.03), (4.0, -3.0, 2.0), T.fixed_centre(shape_xyz))
    lab_m = render_labels(shape_xyz, inv_map=invert(truth))
    moving = intensities(lab_m, (0, 3600, 2000, 1200), rng, 40.0, True, 0, 4095, np.uint16)
    mats = []
    centre = T.fixed_centre(shape_xyz)
    for tx in np.linspace(-10, 10, n_tx):
        for th in np.linspace(-15, 15, n_rot):
            for s in np.linspace(0.9, 1.1, n_scale):
                mats.append(T.centred_matrix(T.affine_matrix((0, 0, th), s), (tx, 0, 0), centre))
    return dict(name="multimodal-sweep 256x256x180 u16", fixed=fixed, moving=moving,
                fixed_range=(0, 4095), moving_range=(0, 4095),
                transforms=np.stack(mats).reshape(-1, 12), bins=128,
                q=[1.0, 0.5, 0.8, 1.2, 1.5, 2.0], truth=truth)


def same_image(shape_xyz=(256, 256, 180), seed: int = 5, dtype=np.uint16) -> dict:
    """One T1-like phantom used as both fixed and moving, the setting of the
    paper's parameter-space maps (the same image on both sides, so the
    optimum is the identity at the map's centre).  u16 levels 0/600/1600/2400
    with Rician noise (sigma 40), range 0..4095, 128 bins; u8 levels
    20/90/160/230 with Gaussian noise (sigma 8), range 0..255, 32 bins.
    Entropies: Shannon and the Tsallis q the paper's maps show."""
    rng = np.random.default_rng(seed)
    lab = render_labels(shape_xyz)
    if np.dtype(dtype) == np.uint8:
        vol = intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.uint8)
        rng_, bins = (0, 255), 32
    else:
        vol = intensities(lab, (0, 600, 1600, 2400), rng, 40.0, True, 0, 4095, np.uint16)
        rng_, bins = (0, 4095), 128
    return dict(name=f"same-image {shape_xyz[0]}x{shape_xyz[1]}x{shape_xyz[2]} {np.dtype(dtype).name}",
                fixed=vol, moving=vol, fixed_range=rng_, moving_range=rng_, bins=bins,
                q=[1.0, 0.5, 0.9, 1.1, 1.5, 2.0])


def random_affines(rng: np.random.Generator, n: int, shape_xyz, rot=10.0, trans=8.0,
                   scale=(0.95, 1.05), shear=0.03) -> np.ndarray:
    mats = [np.zeros((3, 4))][:0]
    for _ in range(n):
        ang = rng.uniform(-rot, rot, 3)
        t = rng.uniform(-trans, trans, 3)
        s = rng.uniform(scale[0], scale[1], 3)
        h = rng.uniform(-shear, shear, 3)
        mats.append(T.centred_matrix(T.affine_matrix(ang, s, h), t, T.fixed_centre(shape_xyz)))
    return np.stack(mats).reshape(-1, 12) if mats else np.zeros((0, 12))


def parzen_gradient(n: int = 128, seed: int = 2, n_transforms: int = 64) -> dict:
    """128^3 f32 phantoms in [0, 1]; moving = fixed under a mild affine;
    Parzen 64 bins, Shannon and q = 1.5; 64 random affines."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    lab = render_labels(shape)
    fixed = (intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0).astype(np.float32)
    truth = T.centred_matrix(T.affine_matrix((3.0, -2.0, 4.0), (1.02, 0.98, 1.01), (0.01, 0.0, -0.01)),
                             (2.5, -1.5, 1.0), T.fixed_centre(shape))
    lab_m = render_labels(shape, inv_map=invert(truth))
    moving = (intensities(lab_m, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.float64) / 255.0).astype(np.float32)
    mats = random_affines(rng, n_transforms, shape)
    return dict(name="parzen-gradient 128^3 f32", fixed=fixed, moving=moving, fixed_range=(0.0, 1.0),
                moving_range=(0.0, 1.0), transforms=mats, bins=64, q=[1.0, 1.5], truth=truth)


EDGES = (64, 96, 128, 160, 192, 256)


def _one_pair(seed_seq, edges) -> dict:
    rng = np.random.default_rng(seed_seq)
    shape = tuple(int(e) for e in rng.choice(edges, 3))
    jit = rng.uniform(0.85, 1.1)
    lab = render_labels(shape, jitter=jit)
    fixed = intensities(lab, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.uint8)
    truth = T.centred_matrix(T.affine_matrix(rng.uniform(-5, 5, 3)), rng.uniform(-4, 4, 3), T.fixed_centre(shape))
    lab_m = render_labels(shape, inv_map=invert(truth), jitter=jit)
    moving = intensities(lab_m, (20, 90, 160, 230), rng, 8.0, False, 0, 255, np.uint8)
    mats = random_affines(rng, 16, shape, rot=10.0, trans=8.0, scale=(1.0, 1.0), shear=0.0)
    return dict(fixed=fixed, moving=moving, transforms=mats)


def uneven_pairs(n_pairs: int = 256, seed: int = 3, per_pair: int = 16, edges=EDGES,
                 threads: int = 0) -> list:
    """Volume pairs with per-axis edge lengths drawn from ``edges``; u8 head
    phantoms with per-pair radius jitter; each pair gets ``per_pair`` rigid
    transforms (angles +-10 deg, translation +-8 voxels); 64 bins.  Pair k
    draws from its own child of SeedSequence(seed), so the result does not
    depend on ``threads`` (0 = one per host core, at most 16)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    seqs = np.random.SeedSequence(seed).spawn(n_pairs)
    if per_pair != 16:
        raise ValueError("per_pair is fixed at 16 by the workload")
    workers = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda sq: _one_pair(sq, edges), seqs))


def ct_mr_pair(fixed_shape=(512, 512, 300), moving_shape=(256, 256, 256), seed: int = 4) -> dict:
    """CT-like i16 fixed (air -1000, brain parenchyma 40 HU and CSF spaces
    10 HU, both +N(0, 20), skull 700..1500 HU, 1 mm) against an MR-like u16
    moving volume of the same anatomy at 2 mm spacing; 256 bins; Tsallis
    q = 1.3 Parzen.  The CSF spaces (ventricles, an off-axis lesion) and the
    FEATURES spheres (CT 400 HU, MR 200) give the CT internal structure that
    pins down all 12 affine parameters."""
    rng = np.random.default_rng(seed)
    fs, ms = np.array([1.0, 1.0, 1.0]), np.array([2.0, 2.0, 2.0])
    fcen = T.fixed_centre(fixed_shape, fs)
    mcen = (np.asarray(moving_shape) - 1) / 2.0 * ms
    mo = fcen - mcen  # moving origin: same physical centre
    lab_f = render_labels(fixed_shape, lesion=True, scale_xyz=(0.45, 0.45, 0.8), features=True)
    skull_f = render_labels(fixed_shape, lesion=False, scale_xyz=(0.50, 0.50, 0.86))
    fixed = np.full(lab_f.shape, -1000.0)
    fixed[skull_f > 0] = rng.uniform(700, 1500, int((skull_f > 0).sum()))
    brain = lab_f > 0
    ct_level = np.array([-1000.0, 10.0, 40.0, 40.0, 400.0])  # by label
    fixed[brain] = ct_level[lab_f[brain]] + 20.0 * rng.standard_normal(int(brain.sum()))
    fixed = np.clip(np.rint(fixed), -1000, 1500).astype(np.int16)
    # moving voxel index -> fixed voxel index (same physical frame)
    m2f = np.zeros((3, 4))
    m2f[:, :3] = np.diag(ms / fs)
    m2f[:, 3] = mo / fs
    lab_m = render_labels(moving_shape, inv_map=m2f, lesion=True, scale_xyz=(0.45, 0.45, 0.8),
                          anatomy_shape_xyz=fixed_shape, features=True)
    skull_m = render_labels(moving_shape, inv_map=m2f, lesion=False, scale_xyz=(0.50, 0.50, 0.86),
                            anatomy_shape_xyz=fixed_shape)
    lev = np.array([0.0, 800.0, 1500.0, 2200.0, 200.0])
    s = np.where(skull_m > 0, 300.0, 0.0)
    s = np.where(lab_m > 0, lev[lab_m], s)
    n1 = rng.standard_normal(s.shape)
    n2 = rng.standard_normal(s.shape)
    moving = np.clip(np.rint(np.sqrt((s + 40 * n1) ** 2 + (40 * n2) ** 2)), 0, 4095).astype(np.uint16)
    return dict(name="ct-mr 512x512x300 i16 vs 256^3 u16", fixed=fixed, moving=moving,
                fixed_range=(-1000, 1500), moving_range=(0, 4095), bins=256, q=[1.3],
                fixed_spacing=tuple(fs), moving_spacing=tuple(ms), moving_origin=tuple(mo),
                start=dict(angles=(0.0, 0.0, 6.0), t=(8.0, -5.0, 4.0), scale=1.04))


def random_volume(rng: np.random.Generator, shape_xyz, dtype, lo, hi) -> np.ndarray:
    """Uniform random integer (or real) volume [nz][ny][nx] in [lo, hi]."""
    nx, ny, nz = shape_xyz
    if np.dtype(dtype).kind == "f":
        return rng.uniform(lo, hi, (nz, ny, nx)).astype(dtype)
    return rng.integers(lo, hi, (nz, ny, nx), endpoint=True).astype(dtype)
