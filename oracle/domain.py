"""Grid over a point cloud's bounding box (test infrastructure).

Paper: Warp-Geo, Sec. 2.3 ("the bounding box of the point cloud" discretised
by a uniform grid of l x m x n cells of size h) and Table 1 / Sec. 3.4 (the
grid density d sets the number of grid points along each coordinate
direction).  The paper gives no formula from d to cell counts; the reading
taken: d cells per unit length, h = 1/d; the box widened by `pad` cells on
every side; each extent rounded up to a multiple of q = 2^L, with L the
fewest halvings that bring the largest extent to 32 or below, and to at least
2q (a multigrid hierarchy that halves every extent then reaches a level of at
most 32 cells per axis with every extent >= 2); the box centred.
"""
from __future__ import annotations

import math

import numpy as np

from .discretize import Grid


def bounding_box(x32):
    """Exact per-axis minimum and maximum of float32 points, as float64."""
    x = np.asarray(x32, np.float32)
    return x.min(axis=0).astype(np.float64), x.max(axis=0).astype(np.float64)


def grid_over_box(lo, hi, density, pad=3):
    """The grid of the reading above for the box [lo, hi]."""
    h = 1.0 / density
    need = [max(math.ceil((hi[a] - lo[a]) / h) + 2 * pad, 1) for a in range(3)]
    L = 0
    while max(need) / 2 ** L > 32:
        L += 1
    q = 2 ** L
    n = tuple(max(math.ceil(need[a] / q), 2) * q for a in range(3))
    glo = tuple(0.5 * (lo[a] + hi[a]) - 0.5 * n[a] * h for a in range(3))
    return Grid(n, glo, h)


def grid_over_cloud(x32, density, pad=3):
    lo, hi = bounding_box(x32)
    return grid_over_box(lo, hi, density, pad)
