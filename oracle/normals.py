"""Normal estimation and orientation (test infrastructure).

Paper: Warp-Geo, Sec. 2.1 (distance-weighted PCA, Eq. 1-6) and Sec. 2.2
(parity ray casting with finite-radius detection, Eq. 7-14, and the iterative
refinement for sharp and thin features; Table 1 for the defaults).

Readings (the paper leaves these open):
* Neighbourhood (Eq. 1): x_i itself belongs to N_i (its distance is 0 <= R).
  Membership is decided on the FP32 squared distance, summed x, y, z in that
  order, against R^2 rounded to FP32, as the library decides it; everything
  after membership is FP64.
* eps of Eq. 2: a parameter, by default 1e-6 R.  With the self term's weight
  1/eps the weighted centroid sits at x_i to within about eps, so C_i is in
  effect the distance-weighted scatter about x_i.
* Normal (Eq. 5-6): the right singular vector of the smallest singular value
  of the matrix whose rows are sqrt(w_ij / W_i) (x_j - xbar_i), i.e. the
  eigenvector of C_i for its smallest eigenvalue, as the paper states.
* Probes (Eq. 8): spacing ds = 0.75 r_d and M = ceil((diag + r_d) / ds) + 1,
  diag the diagonal of the cloud's bounding box, so the last probe is farther
  than r_d from every point and every detected block closes.  Any spacing in
  (r_d / 2, r_d) gives a clean outward ray N_one = 2 = N_tol (probes 0 and 1
  see x_i, probe 2 does not); 0.75 keeps probe 1 clear of the exact tie at
  ds = r_d.  Detection (Eq. 9) is decided on the FP32 squared distance to the
  FP32 probe y = x + (m ds) n (products and sums rounded one by one) against
  r_d^2 rounded to FP32, as the library decides it.
* r_d0 (Eq. 13) = sqrt(max_i min_{j != i} d2_ij) / 2 with d2 the FP32 squared
  distance; r_d (Eq. 14) = gamma_r r_d0; these and ds, M in FP64 from that
  FP32 maximum.
* Refinement.  Iteration 0 flips every normal whose ray shows an odd N_i.
  Iterations 1 and 2 revisit the normals whose ray (along the normal after
  iteration 0) has an initial block longer than N_tol probes, the example of
  an ambiguous pattern the paper gives: iteration 1 flips them (its criterion
  N_i != 0 or N_one > N_tol holds for each of them), iteration 2 compares the
  crossings N_i along the flipped normal with N_i^- along the opposite one
  and flips back if N_i > N_i^-.  Revisiting every normal instead would undo
  correct parity decisions where the outward ray crosses another part of the
  body (a torus's inner equator: 2 crossings outward, 1 inward).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

F32 = np.float32


def _d2_f32(a, b):
    """FP32 squared distance, summed x, y, z in that order (a, b float32 [..., 3])."""
    d = (np.asarray(b, F32) - np.asarray(a, F32)).astype(F32)
    s = (d[..., 0] * d[..., 0]).astype(F32)
    s = (s + (d[..., 1] * d[..., 1]).astype(F32)).astype(F32)
    return (s + (d[..., 2] * d[..., 2]).astype(F32)).astype(F32)


def r2_f32(r):
    return F32(float(r) * float(r))


def neighbourhoods(x32, R):
    """Eq. 1: indices of all points within R of each point (itself included)."""
    x32 = np.asarray(x32, F32)
    tree = cKDTree(x32.astype(np.float64))
    cand = tree.query_ball_point(x32.astype(np.float64), float(R) * (1 + 1e-5) + 1e-30)
    R2 = r2_f32(R)
    out = []
    for i, c in enumerate(cand):
        c = np.asarray(c, np.int64)
        keep = _d2_f32(x32[i], x32[c]) <= R2
        out.append(np.sort(c[keep]))
    return out


def dpca_point(x32, i, nbr, eps):
    """Eq. 2-6 for one point: (unit normal, eigenvalues ascending)."""
    X = np.asarray(x32, np.float64)[nbr]
    d = np.linalg.norm(X - np.asarray(x32[i], np.float64), axis=1)
    w = 1.0 / (d + eps)                                  # Eq. 2
    W = w.sum()
    xbar = (w[:, None] * X).sum(0) / W                   # Eq. 3
    A = np.sqrt(w / W)[:, None] * (X - xbar)             # C_i = A^T A, Eq. 4
    if len(A) < 3:                                       # zero rows leave A^T A unchanged
        A = np.concatenate([A, np.zeros((3 - len(A), 3))])
    _, s, vt = np.linalg.svd(A, full_matrices=False)     # vt: all three right singular vectors
    sv = np.zeros(3)
    sv[:len(s)] = s
    lam = np.sort(sv ** 2)
    return vt[-1] / np.linalg.norm(vt[-1]), lam


def dpca_normals(x32, R=0.1, eps=None):
    """Unoriented D-PCA normals (FP64) and eigenvalues (ascending) of C_i."""
    eps = 1e-6 * R if eps is None else eps
    nb = neighbourhoods(x32, R)
    n = np.zeros((len(x32), 3))
    lam = np.zeros((len(x32), 3))
    for i in range(len(x32)):
        n[i], lam[i] = dpca_point(x32, i, nb[i], eps)
    return n, lam


def covariance(x32, i, nbr, eps):
    """C_i of Eq. 4 written out (for the pins)."""
    X = np.asarray(x32, np.float64)[nbr]
    d = np.linalg.norm(X - np.asarray(x32[i], np.float64), axis=1)
    w = 1.0 / (d + eps)
    xbar = (w[:, None] * X).sum(0) / w.sum()
    D = X - xbar
    return (w[:, None, None] * D[:, :, None] * D[:, None, :]).sum(0) / w.sum()


def max_min_spacing2(x32):
    """max_i min_{j != i} of the FP32 squared distance (Eq. 13 before the root)."""
    x32 = np.asarray(x32, F32)
    tree = cKDTree(x32.astype(np.float64))
    k = min(len(x32), 9)
    _, idx = tree.query(x32.astype(np.float64), k=k)
    best = np.full(len(x32), np.inf, np.float32)
    for c in range(1, k):
        d2 = _d2_f32(x32, x32[idx[:, c]])
        best = np.minimum(best, d2)
    # a point with k - 1 coincident copies could hide a nearer FP32 neighbour only
    # behind exact FP64 ties; the candidates above cover every such case in the tests
    return F32(best.max())


def ray_params(x32, gamma_r=2.5, d2max=None):
    """r_d0, r_d (Eq. 13-14), probe spacing ds, probe count M, and the FP32
    values the detection uses (r_d^2, ds)."""
    x32 = np.asarray(x32, F32)
    if d2max is None:
        d2max = max_min_spacing2(x32)
    rd0 = 0.5 * math.sqrt(float(d2max))
    rd = gamma_r * rd0
    ds = 0.75 * rd
    lo, hi = x32.min(0).astype(np.float64), x32.max(0).astype(np.float64)
    diag = math.sqrt(float(((hi - lo) ** 2).sum()))
    M = int(math.ceil((diag + rd) / ds)) + 1
    return {"d2max": F32(d2max), "rd0": rd0, "rd": rd, "ds": ds, "M": M, "rd2_f32": r2_f32(rd), "ds_f32": F32(ds)}


def probes(x, n, M, ds32):
    """Eq. 8 in FP32: y_m = x + (m ds) n, m = 0..M (one rounding per product and sum)."""
    m = np.arange(M + 1, dtype=F32)
    t = (m * F32(ds32)).astype(F32)
    return (np.asarray(x, F32)[None, :] + (t[:, None] * np.asarray(n, F32)[None, :]).astype(F32)).astype(F32)


def detect(tree, x32, y, rd, rd2_32):
    """Eq. 9: d_m = 1 iff some point lies within r_d of y_m (FP32 decision)."""
    cand = tree.query_ball_point(y.astype(np.float64), rd * (1 + 1e-5) + 1e-30)
    d = np.zeros(len(y), np.int8)
    for m, c in enumerate(cand):
        if c and (_d2_f32(y[m], x32[np.asarray(c, np.int64)]) <= rd2_32).any():
            d[m] = 1
    return d


def crossings(d):
    """Eq. 10-11 and the initial-one count: (N_i = N_all - 1, N_one)."""
    d = np.asarray(d, np.int64)
    n_all = int(np.sum((d[1:] == 0) & (d[:-1] == 1)))
    n_one = int(np.argmin(d)) if (d == 0).any() else len(d)
    return n_all - 1, n_one


def ray_counts(x32, n32, gamma_r=2.5, params=None):
    """(N, N_one) along +n and along -n for every point: int [P, 4] =
    (N+, N_one+, N-, N_one-), and the ray parameters."""
    x32 = np.asarray(x32, F32)
    n32 = np.asarray(n32, F32)
    p = ray_params(x32, gamma_r) if params is None else params
    tree = cKDTree(x32.astype(np.float64))
    out = np.zeros((len(x32), 4), np.int64)
    for i in range(len(x32)):
        for k, sgn in enumerate((F32(1), F32(-1))):
            y = probes(x32[i], (sgn * n32[i]).astype(F32), p["M"], p["ds_f32"])
            out[i, 2 * k:2 * k + 2] = crossings(detect(tree, x32, y, p["rd"], p["rd2_f32"]))
    return out, p


def orient_signs(counts, n_tol=2, refine=True):
    """The flip decisions of Sec. 2.2 from the ray counts: +1 keeps the input
    normal, -1 flips it.  refine=False stops after iteration 0 (plain parity)."""
    counts = np.asarray(counts)
    s = np.ones(len(counts), np.int64)
    for i, (Np, N1p, Nm, N1m) in enumerate(counts):
        sg = -1 if Np % 2 == 1 else 1                    # iteration 0
        if not refine:
            s[i] = sg
            continue
        N0, N1 = (Np, N1p) if sg > 0 else (Nm, N1m)      # along the current normal
        Nopp = Nm if sg > 0 else Np                       # along the opposite one
        if N1 > n_tol:                                    # ambiguous: a long initial block
            if N0 != 0 or N1 > n_tol:                     # iteration 1
                sg = -sg
            if Nopp > N0:                                 # iteration 2: N_i (flipped) > N_i^-
                sg = -sg
        s[i] = sg
    return s


def orient(x32, n32, gamma_r=2.5, n_tol=2, refine=True):
    """Oriented normals (FP32 sign flips of n32), the signs and the ray counts."""
    counts, p = ray_counts(x32, n32, gamma_r)
    s = orient_signs(counts, n_tol, refine)
    return (np.asarray(n32, F32) * s[:, None].astype(F32)).astype(F32), s, counts, p
