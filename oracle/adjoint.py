"""Reverse pass of the reconstruction in float64 (test infrastructure).

Paper: Warp-Geo, Sec. 2.5 "Differentiability", Eq. (35)-(39).  The Poisson
solve is differentiated implicitly: one extra solve with A^T (= A) for the
adjoint variable lambda (Eq. 38), then lambda^T db/dtheta (Eq. 39; dA/dtheta
= 0 because the grid does not move with the cloud, Sec. 2.3 after Eq. 21).
Every other piece is the hand-derived transpose of its forward step.
"""
from __future__ import annotations

import numpy as np

from .discretize import OFFSETS, Grid, gather


def splat_weight_grad(grid: Grid, x32, keys):
    """d alpha_{o,i} / d x_i for the 27 stencil cells: [N,27,3].

    alpha = a~ / S, S = sum a~.  d a~/dx_xi = 0 for the central cell; for the
    others d/dx_xi prod_eta 1/2 (1 - |D_eta|/2) with D = (x - c_o)/h is
    -sign(D_xi)/(4h) prod_{eta != xi} 1/2 (1 - |D_eta|/2)  (sign(0) = 0; the
    max(0, .) of Eq. 25 never clips inside the 3x3x3 stencil).  Cells outside
    the grid carry zero weight and zero derivative."""
    x = np.asarray(x32, np.float64)
    k = np.asarray(keys, np.int64)
    cells = k[:, None, :] + OFFSETS[None]
    inside = np.all((cells >= 0) & (cells < np.asarray(grid.n)), axis=2)
    D = (x[:, None, :] - grid.centres(cells)) / grid.h
    f = 0.5 * (1.0 - np.abs(D) / 2.0)                       # [N,27,3]
    raw = np.prod(f, axis=2)
    centre = np.all(OFFSETS == 0, axis=1)
    raw[:, centre] = 0.5
    raw = np.where(inside, raw, 0.0)
    draw = np.zeros(f.shape)
    for xi in range(3):
        o = [a for a in range(3) if a != xi]
        draw[..., xi] = -np.sign(D[..., xi]) / (4.0 * grid.h) * f[..., o[0]] * f[..., o[1]]
    draw[:, centre, :] = 0.0
    draw = np.where(inside[..., None], draw, 0.0)
    S = raw.sum(axis=1)                                      # [N]
    dS = draw.sum(axis=1)                                    # [N,3]
    return draw / S[:, None, None] - raw[..., None] * dS[:, None, :] / (S ** 2)[:, None, None]


def divergence_T(grid: Grid, lam):
    """Transpose of V -> b = -h^2 D_h V:  g_V = -h^2 D_h^T lam.

    D_h puts +F_f/h into the cell below an interior face f and -F_f/h into the
    cell above, with F_f = (V_below + V_above)/2; so each interior face adds
    (lam_below - lam_above)/(2h) to both of its cells' V derivative."""
    gV = np.zeros((3,) + lam.shape)
    for xi in range(3):
        ax = 2 - xi
        m = lam.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        jump = (lam[tuple(lo)] - lam[tuple(hi)]) / (2.0 * grid.h)
        gV[xi][tuple(lo)] += jump
        gV[xi][tuple(hi)] += jump
    return -grid.h ** 2 * gV


def splat_T(grid: Grid, cells, alpha, dalpha, n32, gV):
    """Transpose of (x, n) -> V_o = h^-3 sum_i alpha_{o,i}(x_i) n_i.
    Returns (g_x [N,3], g_n [N,3])."""
    n = np.asarray(n32, np.float64)
    inside = alpha > 0
    cc = np.where(inside[..., None], cells, 0)
    g = np.stack([gather(gV[d], cc) for d in range(3)], axis=2)     # [N,27,3]
    g = np.where(inside[..., None], g, 0.0)
    s = grid.h ** -3
    g_n = s * np.sum(alpha[..., None] * g, axis=1)
    ndot = np.sum(n[:, None, :] * g, axis=2)                          # [N,27]
    g_x = s * np.sum(dalpha * ndot[..., None], axis=1)
    return g_x, g_n


def scatter(shape, cells, w):
    """Sum w[...] into a zero field at integer cells [..., (i,j,k)]."""
    out = np.zeros(shape)
    np.add.at(out, (cells[..., 2].ravel(), cells[..., 1].ravel(), cells[..., 0].ravel()), w.ravel())
    return out


def mc_vertex_T(chi, c, mesh, tri, bary, p_ijk, d_grid, g_d):
    """Reverse of d(p) = |p - p*| through the Marching Cubes vertices.

    Envelope theorem on Eq. (33): with p* = sum_k beta_k v_k the closest point
    on the argmin triangle, d d / d v_k = -beta_k (p - p*) / d (0 if d = 0).
    Eq. (28): a vertex on the edge q1 -> q2 along axis a moves by eta along a,
    eta = (c - chi1)/(chi2 - chi1), so d eta/d chi1 = (c - chi2)/D^2,
    d eta/d chi2 = -(c - chi1)/D^2, d eta/d c = 1/D with D = chi2 - chi1.
    Returns (g_chi, g_c)."""
    g_chi = np.zeros(chi.shape)
    g_c = 0.0
    sel = (g_d != 0) & (d_grid > 0)
    for idx in np.nonzero(sel)[0]:
        t = tri[idx]
        V = mesh.xyz[t]
        pstar = bary[idx] @ V
        u = (p_ijk[idx] - pstar) / d_grid[idx]
        i, j, k = mesh.cube[t]
        for q in range(3):
            gv = -bary[idx, q] * u * g_d[idx]
            e = mesh.edge[t, q]
            if e < 4:
                a, dy, dz, dx = 0, e & 1, e >> 1, 0
            elif e < 8:
                a, dx, dz, dy = 1, (e - 4) & 1, (e - 4) >> 1, 0
            else:
                a, dx, dy, dz = 2, (e - 8) & 1, (e - 8) >> 1, 0
            c1 = np.array([i + dx, j + dy, k + dz])
            c2 = c1.copy()
            c2[a] += 1
            x1 = chi[c1[2], c1[1], c1[0]]
            x2 = chi[c2[2], c2[1], c2[0]]
            D = x2 - x1
            g_eta = gv[a]
            g_chi[c1[2], c1[1], c1[0]] += g_eta * (c - x2) / D ** 2
            g_chi[c2[2], c2[1], c2[0]] += -g_eta * (c - x1) / D ** 2
            g_c += g_eta / D
    return g_chi, g_c
