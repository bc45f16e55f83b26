"""CPU oracle of the discrete gradient paths on a parameter-space map.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product library
and its Python binding never do.  It shares no code with the GPU path.

Results section: the metric of one transform family is mapped over a 3D
grid of the family's parameters (e.g. 51^3 translations between -25 and
25 mm), and the paths a gradient method takes on that map are traced to the
optimum they reach; the Discussion weighs the entropies by that capture
range.  The paper draws the paths but does not define their discretisation.
The reading followed here (and by the GPU path, written separately):

* a path steps from grid point p to the 26-connected neighbour q of
  steepest rise of sign * f, the rise scaled by the reciprocal step length,
  slope = (sign f(q) - sign f(p)) * w with w = 1, 1/sqrt 2 or 1/sqrt 3 as the
  fp64 values nearest those reciprocals;
* it moves only on a strictly positive slope, so a point with no rising
  neighbour is a local extremum and its own successor;
* among equal slopes the first neighbour in (dz, dy, dx) order, each running
  -1, 0, 1, wins; NaN slopes never win;
* the capture radius is the largest Chebyshev radius r about the centre
  whose points all end at the extremum the centre's own path ends at.

Parity pinned by tests: closed-form maps (a concave bowl with one maximum, two
separated bumps with a bisecting basin boundary, a plateau), descent as the
ascent of the negated map, and an independent brute-force loop on tiny maps.
"""
from __future__ import annotations

import numpy as np

# Reciprocal step lengths: 1, 1/sqrt(2), 1/sqrt(3), nearest fp64 values.
_W = {1: 1.0, 2: float("0.70710678118654752440"), 3: float("0.57735026918962576451")}


def successors(values: np.ndarray, direction: int) -> np.ndarray:
    """Flat index of each grid point's successor along its discrete gradient
    path (the point itself at a local extremum).  ``values`` is [nz][ny][nx]."""
    f = direction * np.asarray(values, dtype=np.float64)
    nz, ny, nx = f.shape
    flat = np.arange(f.size, dtype=np.int64).reshape(f.shape)
    best = np.zeros(f.shape)
    arg = flat.copy()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = abs(dx) + abs(dy) + abs(dz)
                if k == 0:
                    continue
                # points p whose neighbour p + (dz, dy, dx) lies inside the grid
                pz = slice(max(0, -dz), nz - max(0, dz))
                py = slice(max(0, -dy), ny - max(0, dy))
                px = slice(max(0, -dx), nx - max(0, dx))
                qz = slice(max(0, dz), nz - max(0, -dz))
                qy = slice(max(0, dy), ny - max(0, -dy))
                qx = slice(max(0, dx), nx - max(0, -dx))
                with np.errstate(invalid="ignore"):
                    slope = (f[qz, qy, qx] - f[pz, py, px]) * _W[k]
                    better = slope > best[pz, py, px]
                best[pz, py, px] = np.where(better, slope, best[pz, py, px])
                arg[pz, py, px] = np.where(better, flat[qz, qy, qx], arg[pz, py, px])
    return arg.reshape(-1)


def sinks(next_idx: np.ndarray) -> np.ndarray:
    """The extremum each point's path ends at: follow successors until a
    point is its own successor."""
    s = np.asarray(next_idx, dtype=np.int64).copy()
    while True:
        t = next_idx[s]
        if np.array_equal(t, s):
            return s
        s = t


def stats(next_idx: np.ndarray, sink: np.ndarray, shape_zyx, centre_xyz) -> tuple:
    """(number of extrema, extremum of the centre's path, points ending there,
    capture radius)."""
    nz, ny, nx = shape_zyx
    cx, cy, cz = centre_xyz
    c = (cz * ny + cy) * nx + cx
    target = int(sink[c])
    extrema = int(np.count_nonzero(next_idx == np.arange(next_idx.size)))
    basin = int(np.count_nonzero(sink == target))
    z, y, x = np.unravel_index(np.arange(sink.size), (nz, ny, nx))
    cheb = np.maximum(np.abs(x - cx), np.maximum(np.abs(y - cy), np.abs(z - cz)))
    outside = sink != target
    if outside.any():
        radius = int(cheb[outside].min()) - 1
    else:
        radius = int(cheb.max())
    return extrema, target, basin, radius


def map_paths(values: np.ndarray, direction: int, centre_xyz) -> dict:
    """Successors, sinks and capture statistics of a [nz][ny][nx] map."""
    nxt = successors(values, direction)
    snk = sinks(nxt)
    return {"next": nxt, "sink": snk, "stats": stats(nxt, snk, np.shape(values), centre_xyz)}
