"""A plain float64 numpy V-cycle, written from the definition of the Poisson
solver's multigrid preconditioner z = M r (wg_mg_apply):

* one level when every extent is <= 64 (the exact solve below is then the
  whole preconditioner); else levels halve every extent while all are even
  and >= 4 and one exceeds 32;
* pre-smoothing from a zero guess: x = wa rhs, x += wb (rhs - A x);
* residual restricted with R = P^T / 2, P the cell-centred trilinear
  prolongation (3/4, 1/4 per axis; the missing neighbour past a boundary
  mirrors with sign +1 for zero flux, -1 for the Dirichlet test mode);
* coarse correction x += P e, then x += wb (rhs - A x), x += wa (rhs - A x);
* coarsest level: the exact solve (constant mode dropped for zero flux) when
  every extent is <= 64, else 32 weighted-Jacobi sweeps (omega 6/7);
* wa, wb: 1 / (6 lambda_k) at the roots lambda_k of the degree-2 Chebyshev
  polynomial on [0.25, 2].

A is the oracle's 7-point operator and the exact coarse solve the oracle's
spectral solve.  Test infrastructure: the GPU tests compare the library with
it, the CPU tests pin it (symmetry, convergence, exactness on one level).
"""
import math

import numpy as np

from oracle import discretize as D

LO = 0.25
L1 = (2 + LO) / 2 - (2 - LO) / 2 * math.cos(math.pi / 4)
L2 = (2 + LO) / 2 + (2 - LO) / 2 * math.cos(math.pi / 4)
WA, WB = 1 / (6 * L1), 1 / (6 * L2)
OMEGA = 6 / 7


def levels(shape):
    out = [tuple(shape)]
    d = tuple(shape)
    if all(v <= 64 for v in d):
        return out
    while all(v % 2 == 0 and v >= 4 for v in d) and any(v > 32 for v in d):
        d = tuple(v // 2 for v in d)
        out.append(d)
    return out


def prolong_1d(nf, nc, mirror):
    P = np.zeros((nf, nc))
    for f in range(nf):
        i = f // 2
        j = i + 1 if f % 2 else i - 1
        if 0 <= j < nc:
            P[f, i] += 0.75
            P[f, j] += 0.25
        else:
            P[f, i] += 0.75 + 0.25 * mirror
    return P


def sep(mats, u):
    """Apply one matrix per axis to u [nz, ny, nx]; mats = (Mz, My, Mx)."""
    u = np.einsum("Kk,kji->Kji", mats[0], u)
    u = np.einsum("Jj,kji->kJi", mats[1], u)
    return np.einsum("Ii,kji->kjI", mats[2], u)


def diag(shape, bc):
    sign = -1 if bc == "neumann" else 1
    miss = np.zeros(shape)
    for ax, n in enumerate(shape):
        idx = np.arange(n)
        m = (idx == 0).astype(float) + (idx == n - 1).astype(float)
        sh = [1, 1, 1]
        sh[ax] = n
        miss = miss + m.reshape(sh)
    return 6 + sign * miss


def vcycle(lv, l, rhs, bc):
    """Level l of the V-cycle on the hierarchy lv (shapes [nz, ny, nx])."""
    A = lambda v: D.apply_A(v, bc)  # noqa: E731
    if l == len(lv) - 1:
        if all(v <= 64 for v in lv[l]):
            return D.solve(rhs, bc)
        dg = diag(lv[l], bc)
        x = OMEGA * rhs / dg
        for _ in range(31):
            x = x + OMEGA * (rhs - A(x)) / dg
        return x
    mirror = 1 if bc == "neumann" else -1
    P = [prolong_1d(nf, nc, mirror) for nf, nc in zip(lv[l], lv[l + 1])]
    x = WA * rhs
    x = x + WB * (rhs - A(x))
    r = rhs - A(x)
    e = vcycle(lv, l + 1, 0.5 * sep([p.T for p in P], r), bc)
    x = x + sep(P, e)
    x = x + WB * (rhs - A(x))
    x = x + WA * (rhs - A(x))
    return x


def apply(rhs, bc):
    """z = M rhs for rhs [nz, ny, nx] (float64)."""
    rhs = np.asarray(rhs, np.float64)
    return vcycle(levels(rhs.shape), 0, rhs, bc)
