"""The Galerkin system with exact quadrature (test infrastructure).

Paper: Warp-Geo, Sec. 2.3, Eq. (21) (A_po = <grad F_p, grad F_o>) and
Eq. (26) (b_p = sum_i sum_o alpha_oi <grad F_p, F_o n_i>), with F the
trilinear tent of Eq. (17) integrated exactly instead of by vertex quadrature.

Reading at the outer faces (the paper is silent on clipped basis functions):
the same zero-flux reading as the 7-point system (Eq. 19's natural
condition): the basis is mirrored across each outer face, evenly for scalars
and for the directions across a vector component, oddly for a component of V
normal to the face (so it carries no flux through it).  Per axis this gives,
with m = M/h, k = h K and g = G (n cells):

  m: rows (1/6, 2/3, 1/6), first and last diagonal 5/6;
  k: rows (-1, 2, -1), first and last diagonal 1;
  g: g[p, p-1] = 1/2, g[p, p+1] = -1/2, g[0, 0] = -1/2, g[n-1, n-1] = 1/2.

In 3-D, A = k (x) m (x) m + m (x) k (x) m + m (x) m (x) k: in the interior the
27-point stencil {8/3, 0, -1/6, -1/12} (centre, faces, edges, corners), at
the boundary the same stencil with indices clamped to the grid.  The
right-hand side is b = h sum_xi (g along xi, m along the other two) V_xi,
which is the vertex-quadrature b of Eq. (26) when m is replaced by the
identity (the lumped mass), so both systems share their scaling.

The cosine modes of the cell-centred grid diagonalise m and k (mirrored
boundaries): k -> 4 sin^2(theta/2), m -> (2 + cos theta)/3, theta = pi q / n.
So A is singular on constants only and solved exactly by the DCT-II.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .discretize import Grid


def mass_1d(n):
    M = np.zeros((n, n))
    for p in range(n):
        M[p, p] = 2.0 / 3.0
        if p > 0:
            M[p, p - 1] = 1.0 / 6.0
        if p + 1 < n:
            M[p, p + 1] = 1.0 / 6.0
    M[0, 0] = M[n - 1, n - 1] = 5.0 / 6.0
    return M


def stiff_1d(n):
    K = np.zeros((n, n))
    for p in range(n):
        K[p, p] = 2.0
        if p > 0:
            K[p, p - 1] = -1.0
        if p + 1 < n:
            K[p, p + 1] = -1.0
    K[0, 0] = K[n - 1, n - 1] = 1.0
    return K


def deriv_1d(n):
    G = np.zeros((n, n))
    for p in range(n):
        if p > 0:
            G[p, p - 1] = 0.5
        if p + 1 < n:
            G[p, p + 1] = -0.5
    G[0, 0] = -0.5
    G[n - 1, n - 1] += 0.5
    return G


def _along(mat, x, xi):
    """Apply a 1-D matrix along grid axis xi (0 = x) of an [nz, ny, nx] array."""
    ax = 2 - xi
    return np.moveaxis(np.tensordot(mat, x, axes=([1], [ax])), 0, ax)


def apply_A(chi):
    """A chi for A = sum_xi k_xi (x) m (x) m."""
    chi = np.asarray(chi, np.float64)
    nz, ny, nx = chi.shape
    n = (nx, ny, nz)
    out = np.zeros_like(chi)
    for xi in range(3):
        t = chi
        for eta in range(3):
            t = _along(stiff_1d(n[eta]) if eta == xi else mass_1d(n[eta]), t, eta)
        out += t
    return out


def divergence(grid: Grid, V):
    """b = h sum_xi (g along xi, m along the others) V_xi (V: [3, nz, ny, nx])."""
    nz, ny, nx = grid.shape
    n = (nx, ny, nz)
    b = np.zeros(grid.shape)
    for xi in range(3):
        t = np.asarray(V[xi], np.float64)
        for eta in range(3):
            t = _along(deriv_1d(n[eta]) if eta == xi else mass_1d(n[eta]), t, eta)
        b += t
    return grid.h * b


def divergence_T(grid: Grid, lam):
    """Transpose of V -> b: g_V_xi = h (g^T along xi, m along the others) lam."""
    nz, ny, nx = grid.shape
    n = (nx, ny, nz)
    gV = np.zeros((3,) + tuple(grid.shape))
    for xi in range(3):
        t = np.asarray(lam, np.float64)
        for eta in range(3):
            t = _along(deriv_1d(n[eta]).T if eta == xi else mass_1d(n[eta]), t, eta)
        gV[xi] = grid.h * t
    return gV


def eigenvalues(shape):
    """Eigenvalues of A on the separable cosine basis (shape [nz, ny, nx])."""
    khat, mhat = [], []
    for ax, m in enumerate(shape):
        th = np.pi * np.arange(m) / m
        sh = [1, 1, 1]
        sh[ax] = m
        khat.append((4.0 * np.sin(th / 2.0) ** 2).reshape(sh))
        mhat.append(((2.0 + np.cos(th)) / 3.0).reshape(sh))
    return (khat[0] * mhat[1] * mhat[2] + mhat[0] * khat[1] * mhat[2] + mhat[0] * mhat[1] * khat[2])


def solve(b):
    """chi = A^+ b (zero mean) by the orthonormal DCT-II."""
    b = np.asarray(b, np.float64)
    lam = eigenvalues(b.shape)
    bh = scipy.fft.dctn(b, type=2, norm="ortho")
    lam[0, 0, 0] = 1.0
    xh = bh / lam
    xh[0, 0, 0] = 0.0
    return scipy.fft.idctn(xh, type=2, norm="ortho")


def rel_residual(chi, b):
    """||P b - A chi||_2 / ||P b||_2 (P: mean removal)."""
    pb = np.asarray(b, np.float64) - np.mean(b)
    return float(np.linalg.norm(pb - apply_A(chi)) / np.linalg.norm(pb))
