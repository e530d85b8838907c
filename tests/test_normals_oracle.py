"""Pins of the normal-estimation and orientation oracle (Sec. 2.1-2.2) to
closed forms, invariants and brute force (CPU)."""
import math

import numpy as np
import pytest

from oracle import normals as NO
from paper_2609_20964_amd import synth


def test_crossing_counts_of_hand_arrays():
    # Eq. 10-11: transitions 1 -> 0 for m >= 1, minus the initial block; initial ones
    assert NO.crossings([1, 1, 0, 0, 1, 0, 1, 1, 0]) == (2, 2)
    assert NO.crossings([1, 0]) == (0, 1)
    assert NO.crossings([1, 1, 1, 0, 0]) == (0, 3)
    assert NO.crossings([1, 0, 1, 0, 1, 1, 1, 0, 0]) == (2, 1)


def test_covariance_of_a_ring_in_closed_form():
    # x_i at the origin, k points on a circle of radius rho in the xy plane:
    # w = 1/(rho + eps) on the ring, 1/eps at the centre, centroid 0 by symmetry,
    # C = (w_ring / W) (k rho^2 / 2) diag(1, 1, 0)
    k, rho, eps = 12, 0.05, 1e-4
    ang = 2 * np.pi * np.arange(k) / k
    ring = np.stack([rho * np.cos(ang), rho * np.sin(ang), np.zeros(k)], 1)
    x = np.concatenate([np.zeros((1, 3)), ring]).astype(np.float32)
    nb = np.arange(k + 1)
    C = NO.covariance(x, 0, nb, eps)
    X = x.astype(np.float64)
    wr = 1.0 / (np.linalg.norm(X[1:], axis=1) + eps)
    W = 1.0 / eps + wr.sum()
    c = (wr[:, None, None] * X[1:, :, None] * X[1:, None, :]).sum(0) / W
    assert np.allclose(C, c, rtol=1e-12, atol=1e-18)
    # the same in closed form, to the FP32 rounding of the ring
    cf = (1.0 / (rho + eps)) / (1.0 / eps + k / (rho + eps)) * k * rho ** 2 / 2
    assert np.allclose(np.diag(C), [cf, cf, 0.0], rtol=1e-6, atol=1e-12)
    n, lam = NO.dpca_point(x, 0, nb, eps)
    assert abs(abs(n[2]) - 1.0) < 1e-12
    assert lam[0] < 1e-12 * lam[2] and abs(lam[1] - lam[2]) < 1e-6 * lam[2]


def test_planar_patch_gives_the_plane_normal():
    rng = np.random.default_rng(71)
    nrm = np.array([0.3, -0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    u = np.cross(nrm, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    v = np.cross(nrm, u)
    ab = rng.uniform(-0.2, 0.2, (400, 2))
    x = (0.5 + ab[:, :1] * u + ab[:, 1:] * v).astype(np.float32)
    n, lam = NO.dpca_normals(x, R=0.08)
    err = np.abs(np.abs(n @ nrm) - 1.0)
    assert err.max() < 1e-10
    assert (lam[:, 0] < 1e-9 * lam[:, 2]).all()


def test_rotation_and_translation_equivariance():
    rng = np.random.default_rng(72)
    x, _ = synth.sphere(600, radius=0.25, seed=73)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    n0, lam = NO.dpca_normals(x, R=0.1)
    xr = ((x.astype(np.float64) - 0.5) @ Q.T + 0.5 + np.array([0.01, -0.02, 0.03])).astype(np.float32)
    n1, _ = NO.dpca_normals(xr, R=0.1)
    gap = (lam[:, 1] - lam[:, 0]) / lam[:, 2]
    ok = gap > 0.05
    cosang = np.abs(np.sum((n0 @ Q.T) * n1, 1))
    # FP32 rounding of the rotated coordinates moves the normals by ~1e-7 / gap
    assert ok.mean() > 0.9 and (1.0 - cosang[ok]).max() < 1e-8


def test_neighbourhoods_against_brute_force():
    rng = np.random.default_rng(74)
    x = rng.uniform(0, 1, (300, 3)).astype(np.float32)
    R = 0.17
    nb = NO.neighbourhoods(x, R)
    R2 = np.float32(R * R)
    for i in range(len(x)):
        want = [j for j in range(len(x))
                if np.float32(np.float32(np.float32((x[j, 0] - x[i, 0]) * (x[j, 0] - x[i, 0])) +
                                         np.float32((x[j, 1] - x[i, 1]) * (x[j, 1] - x[i, 1]))) +
                              np.float32((x[j, 2] - x[i, 2]) * (x[j, 2] - x[i, 2]))) <= R2]
        assert list(nb[i]) == want
        assert i in want


def test_ray_parameters_of_a_hand_cloud():
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0]], np.float32)
    p = NO.ray_params(x, gamma_r=2.5)
    # nearest spacings 1, 1, 2: r_d0 = 1, r_d = 2.5, ds = 1.875, diag = sqrt 5
    assert p["d2max"] == 4.0 and p["rd0"] == 1.0 and p["rd"] == 2.5 and p["ds"] == 1.875
    assert p["M"] == math.ceil((math.sqrt(5.0) + 2.5) / 1.875) + 1 == 4


def test_detection_against_brute_force():
    rng = np.random.default_rng(75)
    x = rng.uniform(0, 1, (200, 3)).astype(np.float32)
    from scipy.spatial import cKDTree
    tree = cKDTree(x.astype(np.float64))
    y = rng.uniform(-0.1, 1.1, (500, 3)).astype(np.float32)
    rd = 0.06
    d = NO.detect(tree, x, y, rd, NO.r2_f32(rd))
    d2 = NO._d2_f32(y[:, None, :], x[None, :, :])
    assert (d == (d2 <= NO.r2_f32(rd)).any(1)).all()
    assert 0 < d.sum() < len(d)


def _random_signs(n, seed):
    s = np.where(np.random.default_rng(seed).uniform(size=len(n)) < 0.5, -1.0, 1.0)
    return (n * s[:, None]).astype(np.float32)


def test_sphere_normals_all_outward():
    x, n = synth.sphere(2500, radius=0.3, seed=76)
    nn = _random_signs(n, 77)
    out, s, counts, _ = NO.orient(x, nn)
    radial = x.astype(np.float64) - 0.5
    assert (np.sum(out * radial, 1) > 0).all()
    # a convex body: every outward ray leaves at once
    outward = np.where(np.sum(nn * radial, 1) > 0, 0, 2)
    assert (counts[np.arange(len(x)), outward] == 0).all()


def test_torus_inner_equator_keeps_its_parity():
    # outward rays from the inner side cross the far side of the ring (N = 2),
    # inward ones cross the tube once: parity orients both correctly and the
    # refinement leaves them alone (their initial blocks are short).  Rays
    # that graze the far side of the ring within r_d of it count a crossing
    # that is not there (the paper's scenario A) and stay wrong: 3% here.
    x, n = synth.torus(6000, pos_sigma=0.0, ang_sigma_deg=0.0, seeds=(78, 79, 80))
    nn = _random_signs(n, 81)
    out, s, counts, _ = NO.orient(x, nn)
    good = np.sum(out.astype(np.float64) * n, 1) > 0
    assert good.mean() > 0.96
    idx = np.arange(len(x))
    col = np.where(np.sum(nn * n, 1) > 0, 0, 2)          # the column of the outward ray
    Nout, N1out, Nin, N1in = counts[idx, col], counts[idx, col + 1], counts[idx, 2 - col], counts[idx, 3 - col]
    # the inner-equator pattern: two crossings outward, one inward, short blocks
    pat = (Nout == 2) & (Nin == 1) & (N1out <= 2) & (N1in <= 2)
    assert pat.sum() > 100 and good[pat].all()
    # every clean pattern (even outward, odd inward) ends outward
    clean = (Nout % 2 == 0) & (Nin % 2 == 1) & (N1out <= 2) & (N1in <= 2)
    assert clean.mean() > 0.9 and good[clean].all()


def _thin_slab(t, spacing, seed):
    """Points on the six faces of the box [0.1, 0.9]^2 x [0.5 -+ t/2] (a jittered
    lattice of the given spacing on each face) and the outward face normals."""
    rng = np.random.default_rng(seed)
    pts, nrm = [], []
    g = np.arange(0.1 + spacing / 2, 0.9, spacing)
    a, b = np.meshgrid(g, g, indexing="ij")
    a, b = a.ravel(), b.ravel()
    for z, nz in ((0.5 + t / 2, 1.0), (0.5 - t / 2, -1.0)):
        j = rng.uniform(-0.2, 0.2, (len(a), 2)) * spacing
        pts.append(np.stack([a + j[:, 0], b + j[:, 1], np.full(len(a), z)], 1))
        nrm.append(np.tile([0, 0, nz], (len(a), 1)))
    zz = np.arange(0.5 - t / 2 + spacing / 4, 0.5 + t / 2, spacing / 2)
    for axis in (0, 1):
        for c, sg in ((0.1, -1.0), (0.9, 1.0)):
            u, w = np.meshgrid(g, zz, indexing="ij")
            p = np.zeros((u.size, 3))
            p[:, axis] = c
            p[:, 1 - axis] = u.ravel()
            p[:, 2] = w.ravel()
            pts.append(p)
            q = np.zeros((u.size, 3))
            q[:, axis] = sg
            nrm.append(q)
    return np.concatenate(pts).astype(np.float32), np.concatenate(nrm)


def test_thin_slab_needs_the_refinement():
    # slab thinner than the detection reach: an inward ray's first block runs
    # through the other face (scenario C), parity alone keeps it inward
    x, n = _thin_slab(t=0.02, spacing=0.016, seed=82)
    p = NO.ray_params(x)
    assert 0.5 * p["rd"] < 0.02 < 1.25 * p["rd"]
    nn = _random_signs(n, 83)
    big = np.abs(n[:, 2]) > 0.5
    plain, _, counts, _ = NO.orient(x, nn, refine=False)
    refined = NO.orient_signs(counts, refine=True)[:, None] * nn
    frac_plain = (np.sum(plain[big] * n[big], 1) > 0).mean()
    frac_ref = (np.sum(refined[big] * n[big], 1) > 0).mean()
    assert frac_plain < 0.7 and frac_ref == 1.0
    assert (np.sum(refined * n, 1) > 0).mean() > 0.98
