"""Surface extraction, signed distance and sampling in float64 (test infrastructure).

Paper: Warp-Geo, Sec. 2.4 "Surface extraction and signed-distance-field
computation", Eq. (27)-(34).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import native
from .discretize import Grid, gather, trilinear_stencil


@dataclass
class Mesh:
    """Triangles of {chi = c}: cube (i,j,k) [T,3], local edge ids [T,3] and
    vertices [T,3,3] in grid units."""
    cube: np.ndarray
    edge: np.ndarray
    xyz: np.ndarray

    def __len__(self):
        return len(self.cube)


def extract(chi, c):
    """Marching Cubes of chi - c on the dual lattice of cell centres (Eq. 27-28);
    corners with chi < c are inside.  The triangulation rule is applied per cube
    at run time (csrc/mcdist.c)."""
    cube, edge, xyz = native.marching_cubes(chi, c)
    return Mesh(cube, edge, xyz)


def node_coords(nodes_lin, grid: Grid):
    """Integer (i,j,k) of linear node indices (x fastest)."""
    nx, ny, _ = grid.n
    nodes_lin = np.asarray(nodes_lin, np.int64)
    return np.stack([nodes_lin % nx, (nodes_lin // nx) % ny, nodes_lin // (nx * ny)], 1)


def sdf_nodes(grid: Grid, chi, c, mesh: Mesh, nodes_lin=None):
    """phi at cell-centre nodes (Eq. 29-34).

    d = exact distance to the nearest triangle (Eq. 33, brute force over every
    triangle), times h.  Sign (Eq. 30): outside is positive; for grid nodes the
    parity test against the closed mesh reduces to sigma = +1 iff chi >= c,
    because the extracted surface separates exactly the chi >= c corners from
    the chi < c ones.  Returns (phi, argmin triangle, barycentrics of the
    closest point, node coords)."""
    if nodes_lin is None:
        nodes_lin = np.arange(chi.size)
    ijk = node_coords(nodes_lin, grid)
    if len(mesh) == 0:
        d = np.full(len(ijk), np.inf)
        arg = np.full(len(ijk), -1)
        bary = np.zeros((len(ijk), 3))
    else:
        d, arg, bary = native.mesh_distance(ijk.astype(np.float64), mesh.xyz)
    sigma = np.where(gather(chi, ijk) >= c, 1.0, -1.0)
    return sigma * d * grid.h, arg, bary, ijk


def node_gradient(grid: Grid, phi, ijk):
    """Grid gradient of phi at nodes ijk [M,3]: central differences, one-sided
    first order on the boundary cells (the 'grid gradients' of the method)."""
    n = np.asarray(grid.n)
    g = np.zeros((len(ijk), 3))
    for xi in range(3):
        e = np.zeros(3, np.int64)
        e[xi] = 1
        lo = ijk[:, xi] == 0
        hi = ijk[:, xi] == n[xi] - 1
        up = np.where(hi[:, None], ijk, ijk + e)
        dn = np.where(lo[:, None], ijk, ijk - e)
        span = (up[:, xi] - dn[:, xi]).astype(np.float64) * grid.h
        g[:, xi] = (gather(phi, up) - gather(phi, dn)) / span
    return g


def sample(grid: Grid, phi, q32):
    """phi(q) by trilinear interpolation of the node values, and the unit
    normal grad phi / |grad phi| (Sec. 2.4, after Eq. 32) with the gradient
    taken on the grid and interpolated trilinearly; a zero gradient gives a
    zero normal."""
    cells, w, _ = trilinear_stencil(grid, q32)
    val = np.sum(w * gather(phi, cells), axis=1)
    M = len(cells)
    g = node_gradient(grid, phi, cells.reshape(-1, 3)).reshape(M, 8, 3)
    G = np.sum(w[..., None] * g, axis=1)
    norm = np.linalg.norm(G, axis=1, keepdims=True)
    nrm = np.where(norm > 0, G / np.where(norm > 0, norm, 1.0), 0.0)
    return val, nrm
