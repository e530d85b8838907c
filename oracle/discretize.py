"""Discretisation steps of the reconstruction in float64 (test infrastructure).

Paper: Warp-Geo, Sec. 2.3 "GPU-efficient Poisson reconstruction on uniform
grids", Eq. (15)-(26).  Each function states the passage it follows and the
reading taken where the paper is silent.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.fft


@dataclass(frozen=True)
class Grid:
    """Uniform grid of n = (nx, ny, nz) cubic cells of size h starting at lo
    (Sec. 2.3, "Galerkin discretization on uniform Eulerian grid").  The
    unknowns sit at cell centres c_o = lo + (o + 1/2) h (Eq. 16-17: one basis
    function per cell, centred on it)."""
    n: tuple
    lo: tuple
    h: float

    @staticmethod
    def unit(n):
        return Grid((n, n, n), (0.0, 0.0, 0.0), 1.0 / n)

    @property
    def shape(self):            # numpy order [nz, ny, nx]
        return (self.n[2], self.n[1], self.n[0])

    def centres(self, idx):
        """World position of cell centres for integer indices idx[...,3] (i,j,k)."""
        return np.asarray(self.lo) + (np.asarray(idx, np.float64) + 0.5) * self.h


# ---------------------------------------------------------------------------
# binning and the 27-cell weights (Eq. 24-25)
# ---------------------------------------------------------------------------

def cell_keys(grid: Grid, x32):
    """Central cell of each point: k = floor((x - lo) / h) per axis, in float64.

    Sec. 2.3 (right-hand side): the 27-cell stencil surrounds the cell holding
    the point.  A point exactly on a face goes to the upper cell.  Returns
    (k [N,3] int64, inside [N] bool)."""
    x = np.asarray(x32, dtype=np.float64)
    t = (x - np.asarray(grid.lo, np.float64)) / grid.h
    k = np.floor(t).astype(np.int64)
    inside = np.all((k >= 0) & (k < np.asarray(grid.n)), axis=1)
    return k, inside


OFFSETS = np.array(list(itertools.product((-1, 0, 1), repeat=3)), dtype=np.int64)[:, ::-1]
"""The 27 stencil offsets (dx, dy, dz), dx fastest."""


def splat_weights(grid: Grid, x32, keys=None):
    """Normalised weights alpha_{o,i} over the 27 cells around each point.

    Eq. (25): the central cell gets 1/2; any other cell o gets
    prod_xi 1/2 max(0, 1 - |x_xi - c_{o,xi}| / (2h)).  Eq. (24): divide by the
    sum over the stencil.  Reading: cells outside the grid are dropped and the
    weights renormalised over the cells kept.

    ``keys`` overrides the central cells (the frozen-stencil protocol).

    Returns (cells [N,27,3] int64, alpha [N,27] float64; alpha = 0 where the
    cell is outside the grid)."""
    x = np.asarray(x32, dtype=np.float64)
    k = cell_keys(grid, x32)[0] if keys is None else np.asarray(keys, np.int64)
    cells = k[:, None, :] + OFFSETS[None, :, :]
    inside = np.all((cells >= 0) & (cells < np.asarray(grid.n)), axis=2)
    c_o = grid.centres(cells)
    raw = np.prod(0.5 * np.maximum(0.0, 1.0 - np.abs(x[:, None, :] - c_o) / (2.0 * grid.h)), axis=2)
    centre = np.all(OFFSETS == 0, axis=1)
    raw[:, centre] = 0.5
    raw = np.where(inside, raw, 0.0)
    return cells, raw / raw.sum(axis=1, keepdims=True)


def normal_field(grid: Grid, cells, alpha, n32):
    """Splatted normal field at cell centres, Eq. (23) with F_o(c_o) = h^-3:
    V_o = h^-3 sum_i alpha_{o,i} n_i (cells, alpha from splat_weights).
    Returns [3, nz, ny, nx]."""
    nrm = np.asarray(n32, dtype=np.float64)
    nx, ny, nz = grid.n
    lin = cells[..., 0] + nx * (cells[..., 1] + ny * cells[..., 2])
    ok = alpha > 0
    V = np.zeros((3, nz * ny * nx))
    for d in range(3):
        w = (alpha * nrm[:, d:d + 1])[ok] / grid.h ** 3
        V[d] = np.bincount(lin[ok], weights=w, minlength=nz * ny * nx)
    return V.reshape(3, nz, ny, nx)


# ---------------------------------------------------------------------------
# divergence and the 7-point operator (Eq. 20-22, 26; Neumann boundary)
# ---------------------------------------------------------------------------

def _axis(xi):                      # grid axis xi (0=x) -> numpy axis of [nz,ny,nx]
    return 2 - xi


def divergence(grid: Grid, V):
    """b = -h^2 D_h V (Eq. 22/26 under vertex quadrature).

    (D_h V)_i = sum_xi (F_{i+1/2} - F_{i-1/2}) / h with face values
    F_{i+1/2} = (V_i + V_{i+1}) / 2 on interior faces and 0 on the outer faces
    (the homogeneous Neumann condition of the weak form, Eq. 19)."""
    b = np.zeros(grid.shape)
    for xi in range(3):
        ax = _axis(xi)
        v = V[xi]
        m = v.shape[ax]
        F = np.zeros(tuple(m + 1 if a == ax else s for a, s in enumerate(v.shape)))
        sl_int = [slice(None)] * 3
        sl_int[ax] = slice(1, m)
        lo_sl = [slice(None)] * 3
        lo_sl[ax] = slice(0, m - 1)
        hi_sl = [slice(None)] * 3
        hi_sl[ax] = slice(1, m)
        F[tuple(sl_int)] = 0.5 * (v[tuple(lo_sl)] + v[tuple(hi_sl)])
        up = [slice(None)] * 3
        up[ax] = slice(1, m + 1)
        dn = [slice(None)] * 3
        dn[ax] = slice(0, m)
        b += (F[tuple(up)] - F[tuple(dn)]) / grid.h
    return -grid.h ** 2 * b


def apply_A(chi, bc="neumann"):
    """A chi with A = -h^2 L_h, the 7-point stencil of Eq. (21) under vertex
    quadrature: (A chi)_i = sum over the 6 faces of (chi_i - chi_j).

    Neumann (Eq. 19): a face on the domain boundary carries no flux.
    Dirichlet (test mode only): a cell-centred ghost chi_g = -chi_i, so a
    boundary face contributes 2 chi_i."""
    chi = np.asarray(chi, np.float64)
    out = np.zeros_like(chi)
    for ax in range(3):
        m = chi.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        flux = chi[tuple(hi)] - chi[tuple(lo)]          # on interior faces
        out[tuple(lo)] -= flux
        out[tuple(hi)] += flux
        if bc == "dirichlet":
            first = [slice(None)] * 3
            last = [slice(None)] * 3
            first[ax] = slice(0, 1)
            last[ax] = slice(m - 1, m)
            out[tuple(first)] += 2.0 * chi[tuple(first)]
            out[tuple(last)] += 2.0 * chi[tuple(last)]
    return out


def eigenvalues(shape, bc="neumann"):
    """Eigenvalues of A on the separable cosine (Neumann) or sine (Dirichlet)
    basis: lambda_k = sum_xi 4 sin^2(k_xi pi / (2 n_xi)), with k from 0..n-1
    (cosine) or 1..n (sine)."""
    lam = np.zeros(shape)
    for ax, m in enumerate(shape):
        k = np.arange(m) if bc == "neumann" else np.arange(1, m + 1)
        l1 = 4.0 * np.sin(k * np.pi / (2.0 * m)) ** 2
        sh = [1, 1, 1]
        sh[ax] = m
        lam = lam + l1.reshape(sh)
    return lam


def solve(b, bc="neumann"):
    """chi = A^+ b exactly by diagonalising A with the orthonormal DCT-II
    (Neumann) or DST-II (Dirichlet); for Neumann the constant mode is set to 0,
    so the result has zero mean (Eq. 20 has constants as its null space).

    The paper solves Eq. (20) iteratively (Sec. 2.5); this direct solve reaches
    the same discrete solution without a tolerance."""
    b = np.asarray(b, np.float64)
    lam = eigenvalues(b.shape, bc)
    if bc == "neumann":
        bh = scipy.fft.dctn(b, type=2, norm="ortho")
        lam[0, 0, 0] = 1.0
        xh = bh / lam
        xh[0, 0, 0] = 0.0
        return scipy.fft.idctn(xh, type=2, norm="ortho")
    bh = scipy.fft.dstn(b, type=2, norm="ortho")
    return scipy.fft.idstn(bh / lam, type=2, norm="ortho")


def project_mean(v):
    """Remove the mean (the Neumann compatibility projection)."""
    return v - np.mean(v)


def rel_residual(chi, b, bc="neumann"):
    """||P b - A chi||_2 / ||P b||_2 in float64 (P = mean removal for Neumann)."""
    b = np.asarray(b, np.float64)
    if bc == "neumann":
        b = project_mean(b)
    r = b - apply_A(chi, bc)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def cg(b, tol=1e-14, maxiter=20000, bc="neumann"):
    """Plain conjugate gradients on A chi = P b (no preconditioner), used only
    to cross-check the direct solve."""
    b = project_mean(b) if bc == "neumann" else np.asarray(b, np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r)
    nb = np.sqrt(rr)
    for _ in range(maxiter):
        q = apply_A(p, bc)
        a = rr / np.vdot(p, q)
        x += a * p
        r -= a * q
        rr2 = np.vdot(r, r)
        if np.sqrt(rr2) <= tol * nb:
            break
        p = r + (rr2 / rr) * p
        rr = rr2
    return project_mean(x) if bc == "neumann" else x


# ---------------------------------------------------------------------------
# trilinear interpolation and the iso-value (Eq. 16; Sec. 2.4)
# ---------------------------------------------------------------------------

def trilinear_stencil(grid: Grid, q32):
    """Corner cells and weights of trilinear interpolation of a cell-centred
    field at points q (Eq. 16 with the trilinear tent as F).

    Continuous index u = (q - lo)/h - 1/2, clamped to [0, n-1]; base cell
    i0 = min(floor(u), n-2); t = u - i0.  Returns (cells [M,8,3], w [M,8],
    dw [M,8,3] = d w / d q, zero on clamped axes)."""
    q = np.asarray(q32, dtype=np.float64)
    n = np.asarray(grid.n)
    u_raw = (q - np.asarray(grid.lo)) / grid.h - 0.5
    u = np.clip(u_raw, 0.0, n - 1.0)
    clamped = (u_raw < 0.0) | (u_raw > n - 1.0)
    i0 = np.minimum(np.floor(u).astype(np.int64), n - 2)
    t = u - i0
    corners = np.array(list(itertools.product((0, 1), repeat=3)), dtype=np.int64)[:, ::-1]
    cells = i0[:, None, :] + corners[None]
    fac = np.where(corners[None] == 1, t[:, None, :], 1.0 - t[:, None, :])   # [M,8,3]
    w = np.prod(fac, axis=2)
    dfac = np.where(corners[None] == 1, 1.0, -1.0) / grid.h * (~clamped[:, None, :])
    dw = np.zeros(fac.shape)
    for xi in range(3):
        others = [a for a in range(3) if a != xi]
        dw[..., xi] = dfac[..., xi] * fac[..., others[0]] * fac[..., others[1]]
    return cells, w, dw


def gather(field, cells):
    """field[k,j,i] at integer cells [..., (i,j,k)]."""
    return field[cells[..., 2], cells[..., 1], cells[..., 0]]


def interp(grid: Grid, field, q32):
    cells, w, _ = trilinear_stencil(grid, q32)
    return np.sum(w * gather(field, cells), axis=1)


def iso_value(grid: Grid, chi, x32):
    """c = mean over the input points of chi_h(x_i) (Sec. 2.4, following the
    standard Poisson-reconstruction choice the paper cites: the average of the
    indicator at the samples)."""
    return float(np.mean(interp(grid, chi, x32)))
