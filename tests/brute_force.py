"""Exact rational brute force of the hard-binned joint histogram.

An independent formulation of the same rules the oracle implements with
128-bit integers: here every quantity is a ``fractions.Fraction``.  The
transform is quantised with Python's round-half-even on the exact rational
value of ``M * 2^32``; the moving coordinate is that rational divided by
2^32; the trilinear weight per axis is the fraction truncated to 16 bits;
the interpolated intensity is the exact weighted sum; the bin is the floor
of ``value * B / R``.  Only suitable for tiny volumes.
"""
from __future__ import annotations

from fractions import Fraction
from math import floor

import numpy as np

TWO32 = 2 ** 32
TWO16 = 2 ** 16


def quantize(M) -> list | None:
    M = np.asarray(M, dtype=np.float64).reshape(12)
    out = []
    for e, m in enumerate(M):
        lim = 2 ** 24 if e % 4 == 3 else 2 ** 16
        if not np.isfinite(m) or abs(m) > lim:
            return None
        out.append(round(Fraction(float(m)) * TWO32))
    return out


def coords(Mq, i, j, k) -> list[Fraction]:
    x = (i, j, k, 1)
    return [Fraction(sum(Mq[4 * r + c] * x[c] for c in range(4)), TWO32) for r in range(3)]


def hist_exact(fixed: np.ndarray, moving: np.ndarray, M, bins: int, frange, mrange,
               clamp: bool = False, keep=None) -> tuple[np.ndarray, int]:
    """Joint histogram [bins][bins] and overlap count, exactly; ``keep``
    ([nz][ny][nx] booleans) limits it to a subset of the fixed voxels."""
    flo, fhi = int(frange[0]), int(frange[1])
    mlo, mhi = int(mrange[0]), int(mrange[1])
    Rf, Rm = fhi - flo + 1, mhi - mlo + 1
    nz, ny, nx = fixed.shape
    mz, my, mx = moving.shape
    mn = (mx, my, mz)
    h = np.zeros((bins, bins), dtype=np.int64)
    Mq = quantize(M)
    if Mq is None:
        return h, -1
    n = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if keep is not None and not keep[k, j, i]:
                    continue
                y = coords(Mq, i, j, k)
                inside = all(0 <= y[r] <= mn[r] - 1 for r in range(3))
                if not inside:
                    if not clamp:
                        continue
                    y = [min(max(y[r], Fraction(0)), Fraction(mn[r] - 1)) for r in range(3)]
                base = [floor(y[r]) for r in range(3)]
                wts = [Fraction(floor((y[r] - base[r]) * TWO16), TWO16) for r in range(3)]
                val = Fraction(0)
                for c in range(8):
                    up = [(c >> r) & 1 for r in range(3)]
                    idx = [min(base[r] + up[r], mn[r] - 1) for r in range(3)]
                    w = Fraction(1)
                    for r in range(3):
                        w *= wts[r] if up[r] else 1 - wts[r]
                    v = int(moving[idx[2], idx[1], idx[0]])
                    v = min(max(v, mlo), mhi) - mlo
                    val += v * w
                bm = floor(val * bins / Rm)
                u = min(max(int(fixed[k, j, i]), flo), fhi) - flo
                bf = floor(Fraction(u * bins, Rf))
                h[bf, bm] += 1
                n += 1
    return h, n
