"""Pins of the oracle's discrete gradient paths on parameter-space maps
(Results: gradient paths on the translation / rotation / scale maps;
Discussion: capture range): hand-worked fixtures, closed-form maps and an
independent brute-force loop on tiny maps."""
import json
import math
import os
import zlib

import numpy as np
import pytest

from oracle import paths as OP

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paths_hand.json")


def brute_force(values, direction, centre):
    """The path rule written as plain loops (no shifted slices)."""
    f = direction * np.asarray(values, dtype=np.float64)
    nz, ny, nx = f.shape
    inv = {1: 1.0, 2: 1.0 / math.sqrt(2.0), 3: 1.0 / math.sqrt(3.0)}
    nxt = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                best, arg = 0.0, (z * ny + y) * nx + x
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            k = abs(dx) + abs(dy) + abs(dz)
                            zz, yy, xx = z + dz, y + dy, x + dx
                            if k == 0 or not (0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx):
                                continue
                            s = (f[zz, yy, xx] - f[z, y, x]) * inv[k]
                            if s > best:
                                best, arg = s, (zz * ny + yy) * nx + xx
                nxt.append(arg)
    sink = []
    for p in range(len(nxt)):
        q = p
        while nxt[q] != q:
            q = nxt[q]
        sink.append(q)
    cx, cy, cz = centre
    target = sink[(cz * ny + cy) * nx + cx]
    radius = None
    far = 0
    for p in range(len(nxt)):
        z, r = divmod(p, ny * nx)
        y, x = divmod(r, nx)
        d = max(abs(x - cx), abs(y - cy), abs(z - cz))
        far = max(far, d)
        if sink[p] != target:
            radius = d - 1 if radius is None else min(radius, d - 1)
    stats = (sum(nxt[p] == p for p in range(len(nxt))), target, sink.count(target),
             far if radius is None else radius)
    return np.array(nxt), np.array(sink), stats


def test_reciprocal_lengths_are_the_nearest_doubles():
    assert OP._W[2] == 1.0 / math.sqrt(2.0) or abs(OP._W[2] - 1.0 / math.sqrt(2.0)) <= 2 ** -53
    assert abs(OP._W[3] - 1.0 / math.sqrt(3.0)) <= 2 ** -53
    # nearest: the neighbouring doubles are farther from the true value
    from fractions import Fraction
    for k, w in ((2, OP._W[2]), (3, OP._W[3])):
        err = abs(Fraction(w) ** 2 * k - 1)
        for nb in (np.nextafter(w, 0.0), np.nextafter(w, 1.0)):
            assert abs(Fraction(float(nb)) ** 2 * k - 1) > err


def test_hand_worked_cases():
    for case in json.load(open(GOLDEN))["cases"]:
        r = OP.map_paths(np.array(case["values_zyx"]), case["direction"], case["centre_xyz"])
        assert r["next"].tolist() == case["next"], case["name"]
        assert r["sink"].tolist() == case["sink"], case["name"]
        assert list(r["stats"]) == case["stats"], case["name"]


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 6), (1, 4, 5), (3, 4, 5), (5, 3, 2)])
@pytest.mark.parametrize("kind", ["noise", "ties", "nan"])
@pytest.mark.parametrize("direction", [1, -1])
def test_matches_brute_force(shape, kind, direction):
    rng = np.random.default_rng(zlib.crc32(repr((shape, kind, direction)).encode()))
    if kind == "noise":
        v = rng.normal(size=shape)
    else:
        v = rng.integers(0, 3, size=shape).astype(np.float64)
        if kind == "nan":
            v[rng.random(shape) < 0.2] = np.nan
    nz, ny, nx = shape
    centre = (nx // 2, ny // 2, nz // 2)
    r = OP.map_paths(v, direction, centre)
    nxt, sink, stats = brute_force(v, direction, centre)
    assert np.array_equal(r["next"], nxt)
    assert np.array_equal(r["sink"], sink)
    assert tuple(r["stats"]) == stats


def test_concave_bowl_has_one_extremum_that_captures_everything():
    nz, ny, nx = 5, 7, 9
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = (6, 2, 1)  # bowl centre (x, y, z), off the grid centre
    f = -(1.0 * (x - c[0]) ** 2 + 1.7 * (y - c[1]) ** 2 + 0.6 * (z - c[2]) ** 2)
    r = OP.map_paths(f, 1, c)
    top = (c[2] * ny + c[1]) * nx + c[0]
    assert np.all(r["sink"] == top)
    n_ext, target, basin, radius = r["stats"]
    assert (n_ext, target, basin) == (1, top, f.size)
    assert radius == max(c[0], nx - 1 - c[0], c[1], ny - 1 - c[1], c[2], nz - 1 - c[2])
    # every step rises strictly
    flat = f.reshape(-1)
    moved = r["next"] != np.arange(f.size)
    assert np.all(flat[r["next"][moved]] > flat[moved])


def test_two_bumps_split_at_the_bisector():
    nz, ny, nx = 5, 5, 21
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a, b = np.array([4, 2, 2]), np.array([16, 2, 2])
    da = (x - a[0]) ** 2 + (y - a[1]) ** 2 + (z - a[2]) ** 2
    db = (x - b[0]) ** 2 + (y - b[1]) ** 2 + (z - b[2]) ** 2
    f = np.exp(-da / 18.0) + np.exp(-db / 18.0)
    r = OP.map_paths(f, 1, tuple(a))
    ia = (a[2] * ny + a[1]) * nx + a[0]
    ib = (b[2] * ny + b[1]) * nx + b[0]
    sink = r["sink"].reshape(nz, ny, nx)
    assert np.all(sink[:, :, :10] == ia) and np.all(sink[:, :, 11:] == ib)
    n_ext, target, basin, radius = r["stats"]
    assert n_ext == 2 and target == ia
    mid_to_a = bool(np.all(sink[:, :, 10] == ia))
    assert radius == (6 if mid_to_a else 5)


def test_plateau_every_point_is_an_extremum():
    f = np.full((3, 4, 5), 2.5)
    r = OP.map_paths(f, 1, (2, 1, 1))
    assert np.array_equal(r["next"], np.arange(f.size))
    assert tuple(r["stats"]) == (f.size, (1 * 4 + 1) * 5 + 2, 1, 0)


def test_descent_is_ascent_of_the_negated_map():
    rng = np.random.default_rng(7)
    f = rng.normal(size=(6, 5, 4))
    a = OP.map_paths(f, -1, (1, 2, 3))
    b = OP.map_paths(-f, 1, (1, 2, 3))
    assert np.array_equal(a["next"], b["next"]) and tuple(a["stats"]) == tuple(b["stats"])
