"""Pins of the FP64 oracle against closed forms, invariants and brute force.

Each test ties an oracle function to something other than itself: hand-derived
values (tests/golden), exact discrete eigen-solutions, affine-field identities,
topological invariants of the extracted mesh, dense brute-force sampling of a
triangle, independent automatic differentiation and finite differences.
"""
import itertools
import os

import numpy as np
import pytest

from oracle import adjoint as A
from oracle import discretize as D
from oracle import native
from oracle import pipeline as P
from oracle import surface as S
from paper_2609_20964_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


# ---------------------------------------------------------------------------
# binning (exact integers)
# ---------------------------------------------------------------------------

def test_cell_keys_exact_on_faces_and_random():
    g = D.Grid.unit(32)
    # x = k/n exactly is a face: goes to the upper cell k
    k = np.arange(32)
    x = np.stack([k / 32.0, (k[::-1]) / 32.0, np.full(32, 0.5)], 1).astype(np.float32)
    keys, inside = D.cell_keys(g, x)
    assert inside.all()
    assert (keys[:, 0] == k).all() and (keys[:, 1] == k[::-1]).all() and (keys[:, 2] == 16).all()
    # power-of-two n on the unit cube: floor(x * n) is exact in binary floating point
    rng = np.random.default_rng(0)
    xr = rng.random((10000, 3)).astype(np.float32)
    keys, _ = D.cell_keys(g, xr)
    assert (keys == np.floor(xr.astype(np.float64) * 32).astype(np.int64)).all()
    # outside points are flagged
    _, inside = D.cell_keys(g, np.array([[1.0, 0.5, 0.5], [-1e-7, 0.5, 0.5]], np.float32))
    assert not inside.any()


# ---------------------------------------------------------------------------
# splat weights (Eq. 24-25)
# ---------------------------------------------------------------------------

def test_splat_weights_hand_values():
    gv = _golden("splat_weights.txt")
    g = D.Grid.unit(8)
    x = np.array([[(3 + 0.5) / 8, (4 + 0.5) / 8, (2 + 0.5) / 8]])
    cells, alpha = D.splat_weights(g, x)
    centre = np.all(D.OFFSETS == 0, axis=1)
    assert alpha[0, centre][0] == pytest.approx(gv["alpha_centre_at_centre"], rel=1e-15)
    face = np.sum(np.abs(D.OFFSETS), axis=1) == 1
    assert np.allclose(alpha[0, face], gv["alpha_face_at_centre"], rtol=1e-15)
    assert alpha.sum() == pytest.approx(1.0, abs=1e-15)
    assert 0.5 / alpha[0, centre][0] == pytest.approx(gv["raw_sum_at_centre"], rel=1e-15)


def test_splat_weights_face_jump():
    gv = _golden("splat_weights.txt")
    g = D.Grid.unit(8)
    yz = (4 + 0.5) / 8
    eps = 1e-12
    before = np.array([[4.0 / 8 - eps, yz, yz]])       # in cell 3, at its upper x face
    after = np.array([[4.0 / 8 + eps, yz, yz]])        # in cell 4
    c0, a0 = D.splat_weights(g, before)
    c1, a1 = D.splat_weights(g, after)
    target = np.array([4, 4, 4])
    w0 = a0[0, np.all(c0[0] == target, axis=1)][0]
    w1 = a1[0, np.all(c1[0] == target, axis=1)][0]
    assert w0 == pytest.approx(gv["alpha_neighbour_before_face"], abs=1e-10)
    assert w1 == pytest.approx(gv["alpha_centre_after_face"], abs=1e-10)
    assert w1 - w0 == pytest.approx(gv["face_jump"], abs=1e-10)


def test_splat_weights_symmetry_and_boundary_renormalisation():
    g = D.Grid.unit(8)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.2, 0.8, (200, 3))
    cells, a = D.splat_weights(g, x)
    assert np.allclose(a.sum(1), 1.0, atol=1e-14)
    # mirror about the grid's centre plane x = 1/2 maps weights onto mirrored cells
    xm = x.copy()
    xm[:, 0] = 1.0 - x[:, 0]
    cm, am = D.splat_weights(g, xm)
    mirror = np.stack([7 - cells[..., 0], cells[..., 1], cells[..., 2]], -1)
    for i in range(len(x)):
        if np.any(np.abs(x[i, 0] * 8 - np.round(x[i, 0] * 8)) < 1e-9):
            continue
        d1 = {tuple(c): w for c, w in zip(mirror[i], a[i])}
        d2 = {tuple(c): w for c, w in zip(cm[i], am[i])}
        for k in d1:
            assert d1[k] == pytest.approx(d2[k], abs=1e-13)
    # a point in a corner cell drops the outside cells and still sums to one
    c, a = D.splat_weights(g, np.array([[0.01, 0.01, 0.99]]))
    assert a.sum() == pytest.approx(1.0)
    assert (a[0] > 0).sum() == 8


def test_splat_weight_gradient_vs_autograd_and_fd():
    torch = pytest.importorskip("torch")
    g = D.Grid.unit(8)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.05, 0.95, (50, 3))
    keys, _ = D.cell_keys(g, x)
    dal = A.splat_weight_grad(g, x, keys)
    # independent: torch autograd of Eq. 24-25 evaluated in float64
    xt = torch.tensor(x, requires_grad=True)
    cells = torch.tensor(keys[:, None, :] + D.OFFSETS[None])
    inside = ((cells >= 0) & (cells < 8)).all(-1)
    c_o = (cells.double() + 0.5) / 8
    raw = (0.5 * (1 - (xt[:, None, :] - c_o).abs() / (2 / 8))).prod(-1)
    centre = torch.tensor(np.all(D.OFFSETS == 0, axis=1))
    raw = torch.where(centre[None], torch.full_like(raw, 0.5), raw)
    raw = torch.where(inside, raw, torch.zeros_like(raw))
    alpha = raw / raw.sum(1, keepdim=True)
    for o in range(27):
        for d in range(3):
            gr = torch.autograd.grad(alpha[:, o].sum(), xt, retain_graph=True)[0][:, d].numpy()
            assert np.allclose(gr, dal[:, o, d], rtol=1e-10, atol=1e-10)
    # central finite differences inside the cell (keys frozen)
    eps = 1e-7
    for d in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, d] += eps
        xm[:, d] -= eps
        _, ap = D.splat_weights(g, xp, keys)
        _, am = D.splat_weights(g, xm, keys)
        assert np.allclose((ap - am) / (2 * eps), dal[..., d], atol=1e-6)


# ---------------------------------------------------------------------------
# normal field and divergence (Eq. 23, 26)
# ---------------------------------------------------------------------------

def test_divergence_affine_field_and_compatibility():
    g = D.Grid.unit(12)
    a = np.array([0.7, -1.3, 2.1])
    kk, jj, ii = np.meshgrid(*(np.arange(12),) * 3, indexing="ij")
    pos = np.stack([ii, jj, kk], 0) * g.h + 0.5 * g.h
    V = a[:, None, None, None] * pos + np.array([0.3, 0.1, -0.2])[:, None, None, None]
    b = D.divergence(g, V)
    inner = (slice(1, -1),) * 3
    # central difference of an affine field is exact: b = -h^2 (a_x + a_y + a_z)
    assert np.allclose(b[inner], -g.h ** 2 * a.sum(), rtol=1e-12, atol=0)
    # zero flux through the boundary: sum b telescopes to 0
    assert abs(b.sum()) <= 1e-13 * np.abs(b).max()
    # constant V -> b vanishes in the interior
    bc = D.divergence(g, np.ones((3, 12, 12, 12)))
    assert np.abs(bc[inner]).max() < 1e-15


def test_splat_conserves_normal_mass():
    g = D.Grid.unit(16)
    x, n = synth.sphere(500, seed=5)
    cells, alpha = D.splat_weights(g, x)
    V = D.normal_field(g, cells, alpha, n)
    # alpha sums to one per point, so the total of V is h^-3 sum_i n_i
    assert np.allclose(V.reshape(3, -1).sum(1) * g.h ** 3, n.astype(np.float64).sum(0), atol=1e-10)


# ---------------------------------------------------------------------------
# operator and exact solve (Eq. 20-21)
# ---------------------------------------------------------------------------

def _eig_rows():
    rows = []
    for line in open(os.path.join(GOLD, "poisson_eigen.txt")):
        if line.strip() and not line.startswith("#"):
            bc, n, kx, ky, kz, lam = line.split()
            rows.append((bc, int(n), int(kx), int(ky), int(kz), float(lam)))
    return rows


def _mode(bc, n, k):
    x = (np.arange(n) + 0.5) / n
    f = np.cos if bc == "neumann" else np.sin
    ux, uy, uz = (f(kk * np.pi * x) for kk in k)
    return uz[:, None, None] * uy[None, :, None] * ux[None, None, :]


@pytest.mark.parametrize("row", _eig_rows())
def test_operator_eigen_solutions(row):
    bc, n, kx, ky, kz, lam = row
    u = _mode(bc, n, (kx, ky, kz))
    Au = D.apply_A(u, bc)
    assert np.abs(Au - lam * u).max() <= 1e-13 * max(1.0, lam)
    assert D.eigenvalues((n, n, n), bc)[kz - (bc == "dirichlet"), ky - (bc == "dirichlet"),
                                          kx - (bc == "dirichlet")] == pytest.approx(lam, rel=1e-14)


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_solve_manufactured(bc):
    n = 16
    ks = [(1, 2, 3), (5, 1, 7), (2, 2, 2)]
    u = sum(_mode(bc, n, k) * (i + 1) for i, k in enumerate(ks))
    lam = [D.eigenvalues((n,) * 3, bc)[k[2] - (bc == "dirichlet"), k[1] - (bc == "dirichlet"),
                                       k[0] - (bc == "dirichlet")] for k in ks]
    b = sum(_mode(bc, n, k) * (i + 1) * lam[i] for i, k in enumerate(ks))
    x = D.solve(b, bc)
    assert np.abs(x - u).max() < 1e-13 * np.abs(u).max()


def test_solve_matches_cg_and_is_mean_free():
    g = D.Grid((12, 10, 14), (0, 0, 0), 1 / 14)
    rng = np.random.default_rng(3)
    b = D.project_mean(rng.standard_normal(g.shape))
    x = D.solve(b)
    xc = D.cg(b, tol=1e-15)
    assert abs(x.mean()) < 1e-14 * np.abs(x).max()
    assert np.abs(x - xc).max() < 1e-11 * np.abs(x).max()
    assert D.rel_residual(x, b) < 1e-13


# ---------------------------------------------------------------------------
# trilinear interpolation and iso-value
# ---------------------------------------------------------------------------

def test_trilinear_reproduces_affine_and_iso_shift():
    g = D.Grid((9, 7, 11), (0.1, -0.2, 0.3), 0.05)
    kk, jj, ii = np.meshgrid(np.arange(11), np.arange(7), np.arange(9), indexing="ij")
    a = np.array([0.3, -2.0, 1.1])
    f = a[0] * ii + a[1] * jj + a[2] * kk + 0.7
    rng = np.random.default_rng(4)
    lo = np.array(g.lo) + 0.5 * g.h
    hi = np.array(g.lo) + (np.array(g.n) - 0.5) * g.h
    q = rng.uniform(lo, hi, (500, 3))
    u = (q - np.array(g.lo)) / g.h - 0.5
    assert np.allclose(D.interp(g, f, q), u @ a + 0.7, atol=1e-12)
    _, _, dw = D.trilinear_stencil(g, q)
    cells, _, _ = D.trilinear_stencil(g, q)
    grad = np.sum(dw * D.gather(f, cells)[..., None], axis=1)
    assert np.allclose(grad, a / g.h, atol=1e-9)
    c0 = D.iso_value(g, f, q)
    assert D.iso_value(g, f + 5.0, q) == pytest.approx(c0 + 5.0, abs=1e-12)


# ---------------------------------------------------------------------------
# Marching Cubes rule, distance and sign (Eq. 27-34)
# ---------------------------------------------------------------------------

def _edge_ends(e):
    if e < 4:
        b0 = 2 * (e & 1) + 4 * (e >> 1); return b0, b0 + 1
    if e < 8:
        b0 = ((e - 4) & 1) + 4 * ((e - 4) >> 1); return b0, b0 + 2
    b0 = ((e - 8) & 1) + 2 * ((e - 8) >> 1); return b0, b0 + 4


def test_mc_cases_cut_only_crossing_edges_and_close_up():
    for case in range(256):
        tris = native.mc_case(case)
        inside = [(case >> b) & 1 for b in range(8)]
        crossing = {e for e in range(12) if inside[_edge_ends(e)[0]] != inside[_edge_ends(e)[1]]}
        used = set(tris.ravel().tolist())
        assert used == crossing, case
        # inside each cube every triangle-fan boundary edge between two crossing
        # edges on a common face appears once; interior fan edges twice
        if case in (0, 255):
            assert len(tris) == 0


def _mesh_edges_global(mesh):
    """Global identity of a vertex = (axis, lower corner) of its grid edge."""
    ids = []
    for t in range(len(mesh)):
        i, j, k = mesh.cube[t]
        vs = []
        for e in mesh.edge[t]:
            b0, b1 = _edge_ends(int(e))
            ax = {1: 0, 2: 1, 4: 2}[b1 - b0]
            vs.append((ax, i + (b0 & 1), j + ((b0 >> 1) & 1), k + ((b0 >> 2) & 1)))
        ids.append(vs)
    return ids


def test_mc_mesh_is_closed_with_sphere_topology():
    g = D.Grid.unit(16)
    kk, jj, ii = np.meshgrid(*(np.arange(16),) * 3, indexing="ij")
    r = np.sqrt((ii - 7.3) ** 2 + (jj - 7.9) ** 2 + (kk - 8.2) ** 2)
    rng = np.random.default_rng(5)
    chi = r + 0.4 * rng.standard_normal(r.shape)        # bumpy sphere-like level set
    mesh = S.extract(chi, 5.0)
    tris = _mesh_edges_global(mesh)
    edges = {}
    verts = set()
    for vs in tris:
        verts.update(vs)
        for a, b in ((0, 1), (1, 2), (2, 0)):
            key = tuple(sorted((vs[a], vs[b])))
            edges[key] = edges.get(key, 0) + 1
    assert set(edges.values()) == {2}             # watertight: every edge in two triangles
    chiE = len(verts) - len(edges) + len(tris)    # Euler characteristic = 2 * components
    assert chiE % 2 == 0 and chiE >= 2


def test_point_triangle_distance_brute_force():
    rng = np.random.default_rng(6)
    for _ in range(30):
        T = rng.standard_normal((1, 3, 3))
        if _ < 3:                                   # degenerate (zero area) triangles
            T[0, 2] = T[0, 1] if _ == 0 else 0.5 * (T[0, 0] + T[0, 1])
        p = rng.standard_normal((40, 3)) * 2
        d, arg, bary = native.mesh_distance(p, T)
        # dense barycentric sampling of the triangle bounds the distance from above
        s = np.linspace(0, 1, 301)
        uu, vv = np.meshgrid(s, s)
        m = uu + vv <= 1
        pts = T[0, 0] + uu[m, None] * (T[0, 1] - T[0, 0]) + vv[m, None] * (T[0, 2] - T[0, 0])
        dd = np.min(np.linalg.norm(p[:, None, :] - pts[None], axis=2), axis=1)
        assert np.all(d <= dd + 1e-12)
        assert np.all(d >= dd - 0.02 * np.linalg.norm(T[0, 1] - T[0, 0]) - 0.02 * np.linalg.norm(T[0, 2] - T[0, 0]))
        # the reported closest point is on the triangle and at the reported distance
        assert np.all(bary >= -1e-12) and np.allclose(bary.sum(1), 1.0)
        cp = bary @ T[0]
        assert np.allclose(np.linalg.norm(p - cp, axis=1), d, atol=1e-12)


def test_affine_field_gives_exact_plane_distances():
    g = D.Grid.unit(12)
    kk, jj, ii = np.meshgrid(*(np.arange(12),) * 3, indexing="ij")
    a = np.array([0.31, -0.57, 0.76])
    chi = a[0] * ii + a[1] * jj + a[2] * kk + 0.123
    c = 0.9
    mesh = S.extract(chi, c)
    phi, arg, bary, ijk = S.sdf_nodes(g, chi, c, mesh)
    exact = (ijk @ a + 0.123 - c) / np.linalg.norm(a) * g.h
    # the plane is clipped to the lattice box: keep nodes whose foot point is inside it
    foot = ijk - np.outer((ijk @ a + 0.123 - c) / (a @ a), a)
    ok = np.all((foot >= 0) & (foot <= 11), axis=1)
    assert ok.sum() > 500
    assert np.abs(phi[ok] - exact[ok]).max() < 1e-12


def test_sign_equals_ray_parity_on_closed_mesh():
    g = D.Grid.unit(16)
    x, n = synth.sphere(3000, radius=0.3, seed=7)
    r = P.Recon(g, x, n)
    phi, _, _, ijk = S.sdf_nodes(g, r.chi, r.c, r.mesh)
    inside = native.ray_parity(ijk.astype(np.float64), r.mesh.xyz)
    assert np.all((phi < 0) == inside)


# ---------------------------------------------------------------------------
# whole forward: sphere closed form
# ---------------------------------------------------------------------------

def test_sphere_closed_form():
    g = D.Grid.unit(32)
    x, n = synth.sphere()
    r = P.Recon(g, x, n)
    assert D.rel_residual(r.chi, r.b) < 1e-13
    phi = r.phi_grid()
    kk, jj, ii = np.meshgrid(*(np.arange(32),) * 3, indexing="ij")
    pos = (np.stack([ii, jj, kk], -1) + 0.5) * g.h
    rad = np.linalg.norm(pos - 0.5, axis=-1)
    far = rad > 2 * g.h
    assert np.abs(phi - (rad - 0.3))[far].max() < g.h
    q = synth.uniform_queries(4096, 102)
    val, nrm = r.sample(q)
    rq = np.linalg.norm(q - 0.5, axis=1)
    m = rq > 3 * g.h
    assert np.abs(val - (rq - 0.3))[m].max() < g.h
    cosang = np.sum(nrm * (q - 0.5) / rq[:, None], 1)
    assert np.degrees(np.arccos(np.clip(cosang[m], -1, 1))).max() < 10.0
    assert np.median(np.degrees(np.arccos(np.clip(cosang[m], -1, 1)))) < 1.0


def test_tiny_cloud_every_node_brute_force():
    g = D.Grid.unit(8)
    x, n = synth.sphere(64, radius=0.25, seed=8)
    r = P.Recon(g, x, n)
    phi = r.phi_grid()
    # every node against the dense triangle sampling (independent of the C distance)
    tri = r.mesh.xyz
    s = np.linspace(0, 1, 41)
    uu, vv = np.meshgrid(s, s)
    m = uu + vv <= 1
    pts = (tri[:, None, 0] + uu[m][None, :, None] * (tri[:, None, 1] - tri[:, None, 0])
           + vv[m][None, :, None] * (tri[:, None, 2] - tri[:, None, 0])).reshape(-1, 3)
    kk, jj, ii = np.meshgrid(*(np.arange(8),) * 3, indexing="ij")
    nodes = np.stack([ii, jj, kk], -1).reshape(-1, 3).astype(np.float64)
    dd = np.min(np.linalg.norm(nodes[:, None] - pts[None], axis=2), axis=1)
    assert np.all(np.abs(phi.reshape(-1)) / g.h <= dd + 1e-12)
    assert np.all(np.abs(phi.reshape(-1)) / g.h >= dd - 0.05)


# ---------------------------------------------------------------------------
# adjoint: transposes and the whole chain against frozen-stencil FD
# ---------------------------------------------------------------------------

def test_divergence_transpose():
    g = D.Grid((7, 9, 6), (0, 0, 0), 0.1)
    rng = np.random.default_rng(9)
    V = rng.standard_normal((3,) + g.shape)
    lam = rng.standard_normal(g.shape)
    lhs = np.vdot(D.divergence(g, V), lam)
    rhs = np.vdot(V, A.divergence_T(g, lam))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_splat_transpose_in_normals():
    g = D.Grid.unit(10)
    rng = np.random.default_rng(10)
    x = rng.uniform(0.02, 0.98, (300, 3))
    nrm = rng.standard_normal((300, 3))
    cells, alpha = D.splat_weights(g, x)
    gV = rng.standard_normal((3,) + g.shape)
    V = D.normal_field(g, cells, alpha, nrm)
    _, g_n = A.splat_T(g, cells, alpha, np.zeros(alpha.shape + (3,)), nrm, gV)
    assert np.vdot(V, gV) == pytest.approx(np.vdot(nrm, g_n), rel=1e-12)


def test_trilinear_scatter_transpose():
    g = D.Grid((6, 5, 7), (0, 0, 0), 0.2)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(g.shape)
    q = rng.uniform(0, 1.2, (100, 3))
    y = rng.standard_normal(100)
    cells, w, _ = D.trilinear_stencil(g, q)
    assert np.vdot(D.interp(g, f, q), y) == pytest.approx(np.vdot(f, A.scatter(g.shape, cells, w * y[:, None])), rel=1e-12)


def _small_diff_problem():
    """A 20^3 star-shape problem with 4 Fourier coefficients."""
    torch = pytest.importorskip("torch")
    c0 = np.array([0.03, -0.02, 0.015, 0.01])
    shape = synth.StarShape(c0, semi_axes=(0.3, 0.2, 0.22))
    dirs = synth.unit_sphere_dirs(np.random.default_rng(12), 1500)
    tdirs = synth.unit_sphere_dirs(np.random.default_rng(13), 300)
    tshape = synth.StarShape(c0 + 0.01, semi_axes=(0.3, 0.2, 0.22))
    targets = synth.X0 + tshape.rho(tdirs)[:, None] * tdirs
    return torch, shape, dirs, targets


def _cloud(torch, shape, dirs, c):
    ct = torch.tensor(c, dtype=torch.float64, requires_grad=True)
    x, n = synth.star_points_torch(shape, dirs, ct)
    return ct, x, n


def test_whole_chain_gradient_vs_frozen_fd():
    torch, shape, dirs, targets = _small_diff_problem()
    g = D.Grid.unit(20)
    c0 = shape.coeffs
    ct, x, n = _cloud(torch, shape, dirs, c0)
    xn, nn = x.detach().numpy(), n.detach().numpy()
    L0, r = P.loss_mean_sq(g, xn, nn, targets)
    phi, _ = r.sample(targets)
    g_x, g_n, _ = r.backward(targets, 2.0 * phi / len(targets))
    (grad,) = torch.autograd.grad((x * torch.tensor(g_x)).sum() + (n * torch.tensor(g_n)).sum(), ct)
    grad = grad.numpy()
    keys = r.keys
    eps = 1e-4
    fd = np.zeros_like(c0)
    for j in range(len(c0)):
        vals = []
        for s in (+1, -1):
            c = c0.copy()
            c[j] += s * eps
            _, xx, nn2 = _cloud(torch, shape, dirs, c)
            vals.append(P.loss_mean_sq(g, xx.detach().numpy(), nn2.detach().numpy(), targets, keys=keys)[0])
        fd[j] = (vals[0] - vals[1]) / (2 * eps)
    assert np.linalg.norm(grad - fd) <= 1e-3 * np.linalg.norm(fd) + 1e-12, (grad, fd)


def test_query_gradient_vs_fd():
    g = D.Grid.unit(16)
    x, n = synth.sphere(2000, seed=14)
    r = P.Recon(g, x, n)
    rng = np.random.default_rng(15)
    q = rng.uniform(0.15, 0.85, (40, 3))
    wphi = rng.standard_normal(40)
    wn = rng.standard_normal((40, 3))
    _, _, g_q = r.backward(q, wphi, wn)
    eps = 1e-6

    def L(qq):
        v, nn = r.sample(qq)
        return np.sum(wphi * v) + np.sum(wn * nn)
    fd = np.zeros_like(q)
    for i in range(40):
        for d in range(3):
            qp, qm = q.copy(), q.copy()
            qp[i, d] += eps
            qm[i, d] -= eps
            fd[i, d] = (L(qp) - L(qm)) / (2 * eps)
    assert np.allclose(g_q, fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max())


@pytest.mark.parametrize("exact", [False, True])
def test_whole_chain_gradient_with_normal_term_vs_frozen_fd(exact):
    # exact: the system with exact quadrature (27-point stiffness, consistent right-hand side)
    torch, shape, dirs, targets = _small_diff_problem()
    g = D.Grid.unit(20)
    c0 = shape.coeffs
    wdir = np.random.default_rng(16).standard_normal((len(targets), 3))

    def loss(xn, nn, keys=None):
        r = P.Recon(g, xn, nn, keys=keys, exact=exact)
        phi, nq = r.sample(targets)
        return float(np.mean(phi ** 2) + np.mean(np.sum(wdir * nq, 1))), r, phi

    ct, x, n = _cloud(torch, shape, dirs, c0)
    L0, r, phi = loss(x.detach().numpy(), n.detach().numpy())
    T = len(targets)
    g_x, g_n, _ = r.backward(targets, 2.0 * phi / T, wdir / T)
    (grad,) = torch.autograd.grad((x * torch.tensor(g_x)).sum() + (n * torch.tensor(g_n)).sum(), ct)
    grad = grad.numpy()
    eps = 1e-4
    fd = np.zeros_like(c0)
    for j in range(len(c0)):
        vals = []
        for s in (+1, -1):
            c = c0.copy()
            c[j] += s * eps
            _, xx, nn2 = _cloud(torch, shape, dirs, c)
            vals.append(loss(xx.detach().numpy(), nn2.detach().numpy(), keys=r.keys)[0])
        fd[j] = (vals[0] - vals[1]) / (2 * eps)
    assert np.linalg.norm(grad - fd) <= 2e-3 * np.linalg.norm(fd), (grad, fd)


def test_c3_gradient_at_128_vs_frozen_fd():
    """The differentiable configuration at its own size (16-coefficient
    superellipsoid, 100,000 points, 128^3): the oracle's dL/dc for two
    coefficients against central differences (eps 1e-4) of the oracle forward
    with frozen central cells, at 1000 of the targets."""
    torch = pytest.importorskip("torch")
    case = synth.diff_case(n_targets=1000)
    g = D.Grid.unit(128)
    c0 = case.shape.coeffs

    def cloud(c):
        ct = torch.tensor(c, dtype=torch.float64, requires_grad=True)
        x, n = synth.star_points_torch(case.shape, case.dirs, ct)
        return ct, x, n

    ct, x, n = cloud(c0)
    L0, r = P.loss_mean_sq(g, x.detach().numpy().astype(np.float32), n.detach().numpy().astype(np.float32),
                           case.targets)
    phi, _ = r.sample(case.targets)
    g_x, g_n, _ = r.backward(case.targets, 2.0 * phi / len(case.targets))
    (grad,) = torch.autograd.grad((x * torch.tensor(g_x)).sum() + (n * torch.tensor(g_n)).sum(), ct)
    grad = grad.numpy()
    eps = 1e-4
    for j in (0, 7):
        vals = []
        for s in (+1, -1):
            c = c0.copy()
            c[j] += s * eps
            _, xx, nn = cloud(c)
            vals.append(P.loss_mean_sq(g, xx.detach().numpy().astype(np.float32),
                                       nn.detach().numpy().astype(np.float32), case.targets, keys=r.keys)[0])
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(grad[j] - fd) <= 1e-3 * abs(fd), (j, grad[j], fd)
