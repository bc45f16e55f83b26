"""Parameter-space maps of the metric and the gradient paths on them.

Results (Translation, Rotation, Scale): the metric of one transform family
is evaluated over a 3D grid of that family's parameters -- 51 values per
axis, e.g. translations from -25 to 25 mm, 51^3 = 132651 evaluations -- and
the paths a gradient method follows on each map show which starting points
reach the known optimum (the grid centre for a pair already registered);
the Discussion compares the entropies by that capture range.

Each grid point becomes one candidate 3x4 matrix; one batched ``mi_eval``
per batch of points evaluates them all, every entropy from the same
histogram; ``mi_map_paths`` then traces the discrete gradient paths and the
capture statistics of each entropy's map.  This module builds the matrices
(host-side transform setup, as for every call) and marshals the calls.

Families, as parameters p of the fixed -> moving map T of Fig. 1 about the
fixed volume's physical centre c:

* ``translation``: T(x) = x + p (mm);
* ``rotation``: T(x) = R(p) (x - c) + c, with p the vector part of a unit
  quaternion (a versor): rotation by 2 asin|p| about p / |p|.  Points with
  |p| > 1 are scaled onto the unit sphere, the rotation by 180 degrees about
  p / |p| -- the paper maps every point outside the unit sphere to its
  surface;
* ``scale``: T(x) = diag(1 + p) (x - c) + c.
"""
from __future__ import annotations

import numpy as np

from . import binding as B
from . import transforms as T

FAMILIES = ("translation", "rotation", "scale")
DEFAULT_EXTENT = {"translation": 25.0, "rotation": 1.0, "scale": 0.25}


def versor_matrices(v) -> np.ndarray:
    """Rotation matrices [n][3][3] of versors with vector parts ``v`` [n][3]
    (scaled onto the unit sphere where |v| > 1)."""
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    n2 = np.einsum("ij,ij->i", v, v)
    outside = n2 > 1.0
    v = np.where(outside[:, None], v / np.sqrt(np.where(outside, n2, 1.0))[:, None], v)
    w = np.where(outside, 0.0, np.sqrt(np.clip(1.0 - n2, 0.0, None)))
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    R = np.empty((v.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def family_affines(family: str, p) -> tuple[np.ndarray, np.ndarray]:
    """(A [n][3][3], t [n][3]) of the centred maps T(x) = A (x - c) + c + t
    for parameter rows p [n][3]."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    eye = np.broadcast_to(np.eye(3), (p.shape[0], 3, 3)).copy()
    if family == "translation":
        return eye, p.copy()
    if family == "rotation":
        return versor_matrices(p), np.zeros_like(p)
    if family == "scale":
        return eye * (1.0 + p)[:, None, :], np.zeros_like(p)
    raise ValueError(f"unknown family {family!r}; expected one of {FAMILIES}")


def grid_params(n: int, extent: float) -> np.ndarray:
    """Parameter rows [n^3][3] of the grid, x parameter fastest: row
    (k n + j) n + i holds (g[i], g[j], g[k])."""
    g = grid_axis(n, extent)
    pz, py, px = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([px.reshape(-1), py.reshape(-1), pz.reshape(-1)], axis=1)


def grid_axis(n: int, extent: float) -> np.ndarray:
    """n parameter values from -extent to extent (the centre is 0 for odd n)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    return np.linspace(-extent, extent, n) if n > 1 else np.zeros(1)


def map_transforms(family: str, n: int, fixed_shape_xyz, extent: float | None = None,
                   fixed_spacing=(1.0, 1.0, 1.0), fixed_origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Physical matrices [n^3][12] of the family over an n^3 grid, about the
    fixed volume's physical centre; grid point (i, j, k) -- parameters
    (g[i], g[j], g[k]) -- at row (k n + j) n + i, so a [n][n][n] view of any
    per-transform output is the [z][y][x] map."""
    ext = DEFAULT_EXTENT[family] if extent is None else float(extent)
    A, t = family_affines(family, grid_params(n, ext))
    return T.centred_matrices(A, t, T.fixed_centre(fixed_shape_xyz, fixed_spacing, fixed_origin))


def z_order(n: int) -> np.ndarray:
    """Grid rows (x fastest) in Z order (Morton order of (i, j, k)): runs of
    consecutive rows are compact blocks of the parameter grid."""
    g = np.arange(n ** 3)
    k, r = np.divmod(g, n * n)
    j, i = np.divmod(r, n)
    code = np.zeros_like(g)
    for b in range(int(n - 1).bit_length() if n > 1 else 1):
        code |= (((i >> b) & 1) << (3 * b)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b + 2))
    return np.argsort(code, kind="stable")


def mi_map(ctx, fixed, moving, family: str, n: int = 51, extent: float | None = None, bins: int = 64,
           q=(1.0,), flags: int = 0, batch: int = 16384, transforms=None, sample=None,
           order: str = "auto", compact: str | bool = "auto"):
    """MI maps [n_q][n][n][n] (device float64, [z][y][x] order per q) of one
    family over an n^3 grid: batches of grid points through ``ctx.eval``
    (or, with ``sample`` = (fraction, seed), ``ctx.eval_sampled``: every
    point over the same random subset of fixed voxels, as Mattes' MI
    samples them).  ``transforms`` (the [n^3][12] matrices, on the device)
    may be given to skip building them (by default they are built about the
    fixed volume's physical centre).  ``order`` ("grid", "z" or
    "auto") and ``compact`` (bool or "auto") choose the evaluation order of
    the grid points and the compact-slab sweep; neither changes a value."""
    import torch
    dev = fixed.tensor.device
    if transforms is None:
        nz, ny, nx = fixed.tensor.shape
        transforms = torch.from_numpy(map_transforms(family, n, (nx, ny, nz), extent, fixed.spacing,
                                                     fixed.origin)).to(dev)
    total = n ** 3
    if transforms.shape != (total, 12):
        raise ValueError(f"transforms must be [{total}][12]")
    qs = tuple(float(v) for v in np.atleast_1d(q))
    out = torch.empty((total, len(qs)), dtype=torch.float64, device=dev)
    hard = sample is None and not flags & B.HIST_PARZEN
    # the transforms of a batch run at once: in Z order they are compact
    # blocks of the grid, whose moving footprints overlap in L2 (results are
    # identical; the rows are put back in grid order afterwards).  That pays
    # for rotations on every path, 6-9% sampled or Parzen and more with the
    # compact-slab sweep of the hard path; translations and scales keep
    # nearly the same footprint anyway and run slower in Z order.
    if compact == "auto":
        compact = hard and family == "rotation"
    if order == "auto":
        order = "z" if family == "rotation" else "grid"
    if compact:
        flags |= B.COMPACT_SLABS
    if order == "z":
        order = torch.from_numpy(z_order(n)).to(dev)
        transforms = transforms.index_select(0, order)
        grid_out, out = out, torch.empty_like(out)
    else:
        order = None
    for a in range(0, total, batch):
        b = min(total, a + batch)
        if sample is None:
            ctx.eval(fixed, moving, transforms[a:b], bins, qs, flags=flags, want_overlap=False, out=out[a:b])
        else:
            ctx.eval_sampled(fixed, moving, transforms[a:b], bins, qs, fraction=sample[0], seed=sample[1],
                             flags=flags, want_overlap=False, out=out[a:b])
    if order is not None:
        grid_out.index_copy_(0, order, out)
        out = grid_out
    return out.t().reshape(len(qs), n, n, n).contiguous()


def map_paths(ctx, maps, direction: int = 1, centre=None) -> list[dict]:
    """Discrete gradient paths on each map of ``maps`` ([n_q][nz][ny][nx] or
    one [nz][ny][nx] map): per map, successors, sinks and the statistics
    (extrema, sink of the centre, its basin size, capture radius)."""
    if maps.dim() == 3:
        maps = maps.unsqueeze(0)
    res = []
    for m in maps:
        nxt, sink, stats = ctx.map_paths(m, direction, centre)
        res.append({"next": nxt, "sink": sink, "stats": stats})
    return res
