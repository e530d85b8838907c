"""The whole reconstruction and its reverse pass in float64 (test infrastructure).

Forward (paper Sec. 2.3-2.4): bin points -> 27-cell splat V (Eq. 23-25) ->
b = -h^2 D_h V (Eq. 26) -> chi = A^+ b (Eq. 20) -> iso-value c -> Marching
Cubes mesh (Eq. 27-28) -> phi on grid nodes (Eq. 29-34) -> trilinear sampling
of phi and of its grid gradient.

Reverse (Sec. 2.5, Eq. 35-39): transposed sampling -> distance / vertex
adjoint -> iso-value adjoint -> adjoint solve A lambda = P g_chi ->
transposed divergence -> transposed splat.

phi is computed lazily at the nodes a query set needs (brute-force distance
over every triangle), so large grids stay tractable for sampled checks.
"""
from __future__ import annotations

import numpy as np

from . import adjoint as adj
from . import discretize as D
from . import galerkin as G
from . import surface as S


class Recon:
    """exact=True: the Galerkin system with exact quadrature (oracle/galerkin.py)
    instead of vertex quadrature (the 7-point operator)."""

    def __init__(self, grid: D.Grid, x32, n32, keys=None, bc="neumann", exact=False):
        self.grid = grid
        self.exact = exact
        self.x = np.asarray(x32, np.float64)
        self.n = np.asarray(n32, np.float64)
        k, inside = D.cell_keys(grid, x32)
        if not inside.all():
            raise ValueError("point outside the grid")
        self.keys = k if keys is None else np.asarray(keys, np.int64)
        self.cells, self.alpha = D.splat_weights(grid, x32, self.keys)
        self.V = D.normal_field(grid, self.cells, self.alpha, n32)
        if exact:
            self.b = G.divergence(grid, self.V)
            self.chi = G.solve(self.b)
        else:
            self.b = D.divergence(grid, self.V)
            self.chi = D.solve(self.b)
        self.c = D.iso_value(grid, self.chi, x32)
        self.mesh = S.extract(self.chi, self.c)
        N = int(np.prod(grid.n))
        self.phi = np.full(grid.shape, np.nan)
        self.arg = np.full(N, -1, np.int64)
        self.bary = np.zeros((N, 3))
        self.dist = np.full(N, np.nan)
        self.have = np.zeros(N, bool)

    # -- forward --------------------------------------------------------------
    def phi_nodes(self, lin):
        """phi at linear node indices ``lin`` (in the given order)."""
        lin = np.asarray(lin, np.int64)
        uniq = np.unique(lin)
        todo = uniq[~self.have[uniq]]
        if len(todo):
            phi, arg, bary, _ = S.sdf_nodes(self.grid, self.chi, self.c, self.mesh, todo)
            self.phi.reshape(-1)[todo] = phi
            self.arg[todo] = arg
            self.bary[todo] = bary
            self.dist[todo] = np.abs(phi) / self.grid.h
            self.have[todo] = True
        return self.phi.reshape(-1)[lin]

    def phi_grid(self):
        self.phi_nodes(np.arange(self.phi.size))
        return self.phi

    def needed_nodes(self, q32):
        """Linear indices of the nodes that sampling at q reads: the 8 trilinear
        corners and their gradient neighbours."""
        cells, _, _ = D.trilinear_stencil(self.grid, q32)
        c = cells.reshape(-1, 3)
        n = np.asarray(self.grid.n)
        allc = [c]
        for xi in range(3):
            e = np.zeros(3, np.int64)
            e[xi] = 1
            allc.append(np.clip(c + e, 0, n - 1))
            allc.append(np.clip(c - e, 0, n - 1))
        a = np.concatenate(allc)
        nx, ny, _ = self.grid.n
        return np.unique(a[:, 0] + nx * (a[:, 1] + ny * a[:, 2]))

    def sample(self, q32):
        self.phi_nodes(self.needed_nodes(q32))
        return S.sample(self.grid, self.phi, q32)

    # -- reverse --------------------------------------------------------------
    def backward(self, q32, g_phi_q, g_n_q=None):
        """Gradients of L w.r.t. point positions, point normals and queries,
        given dL/dphi(q) [Q] and optionally dL/dn(q) [Q,3]."""
        g = self.grid
        self.phi_nodes(self.needed_nodes(q32))
        q = np.asarray(q32, np.float64)
        cells, w, dw = D.trilinear_stencil(g, q32)
        M = len(q)
        g_phi_q = np.asarray(g_phi_q, np.float64)
        # B1: transposed sampling of phi(q) ...
        phi_c = D.gather(self.phi, cells)
        g_phi = adj.scatter(g.shape, cells, w * g_phi_q[:, None])
        g_q = np.sum(dw * (phi_c * g_phi_q[:, None])[..., None], axis=1)
        # ... and of n(q) = G/|G|, G = sum_c w_c grad_h(phi)_c
        if g_n_q is not None:
            gn = np.asarray(g_n_q, np.float64)
            nodes = cells.reshape(-1, 3)
            gc = S.node_gradient(g, self.phi, nodes).reshape(M, 8, 3)
            Gs = np.sum(w[..., None] * gc, axis=1)
            nG = np.linalg.norm(Gs, axis=1, keepdims=True)
            nh = Gs / np.where(nG > 0, nG, 1.0)
            gG = np.where(nG > 0, (gn - nh * np.sum(nh * gn, 1, keepdims=True)) / np.where(nG > 0, nG, 1.0), 0.0)
            g_q += np.einsum("mcx,mcy,my->mx", dw, gc, gG)
            g_gc = (w[..., None] * gG[:, None, :]).reshape(-1, 3)       # dL/d grad_c
            n = np.asarray(g.n)
            for xi in range(3):
                e = np.zeros(3, np.int64)
                e[xi] = 1
                lo = nodes[:, xi] == 0
                hi = nodes[:, xi] == n[xi] - 1
                up = np.where(hi[:, None], nodes, nodes + e)
                dn = np.where(lo[:, None], nodes, nodes - e)
                span = (up[:, xi] - dn[:, xi]).astype(np.float64) * g.h
                g_phi += adj.scatter(g.shape, up, g_gc[:, xi] / span)
                g_phi -= adj.scatter(g.shape, dn, g_gc[:, xi] / span)
        # B2: distance and Marching Cubes vertices -> chi, c
        lin = np.nonzero(g_phi.reshape(-1))[0]
        ijk = S.node_coords(lin, g)
        sigma = np.where(D.gather(self.chi, ijk) >= self.c, 1.0, -1.0)
        g_d = sigma * g.h * g_phi.reshape(-1)[lin]
        g_chi, g_c = adj.mc_vertex_T(self.chi, self.c, self.mesh, self.arg[lin], self.bary[lin],
                                     ijk.astype(np.float64), self.dist[lin], g_d)
        # B3: iso-value c = mean_i chi_h(x_i)
        Np = len(self.x)
        pc, pw, pdw = D.trilinear_stencil(g, self.x)
        g_chi += adj.scatter(g.shape, pc, pw * (g_c / Np))
        g_x = (g_c / Np) * np.sum(pdw * D.gather(self.chi, pc)[..., None], axis=1)
        # B4: adjoint solve (A symmetric), Eq. 38
        lam = (G.solve if self.exact else D.solve)(D.project_mean(g_chi))
        # B5, B6: Eq. 39 through b = -h^2 D_h V(x, n) (or its exact-quadrature form)
        gV = G.divergence_T(g, lam) if self.exact else adj.divergence_T(g, lam)
        dalpha = adj.splat_weight_grad(g, self.x, self.keys)
        gx2, g_n = adj.splat_T(g, self.cells, self.alpha, dalpha, self.n, gV)
        self.lam = lam
        self.g_chi = g_chi
        self.g_c = g_c
        return g_x + gx2, g_n, g_q


def loss_mean_sq(grid, x32, n32, targets, keys=None):
    """L = mean_j phi(target_j)^2 (the SDF-matching loss of Eq. 40 with a zero
    target field, evaluated at target points)."""
    r = Recon(grid, x32, n32, keys=keys)
    phi, _ = r.sample(targets)
    return float(np.mean(phi ** 2)), r
