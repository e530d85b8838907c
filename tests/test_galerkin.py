"""The exact-quadrature Galerkin system of the oracle (oracle/galerkin.py),
pinned against brute-force Gauss quadrature of the mirrored trilinear tents,
the hand-derived interior stencil, the vertex-quadrature system it reduces to
with a lumped mass, closed-form eigenpairs and a dense conjugate-gradient
solve."""
import numpy as np
import pytest

from oracle import discretize as D
from oracle import galerkin as G


def _tent(x, c, h):
    return np.maximum(0.0, 1.0 - np.abs(x - c) / h)


def _dtent(x, c, h):
    inside = np.abs(x - c) < h
    return np.where(inside, -np.sign(x - c) / h, 0.0)


def _quad_1d(n, h=0.37):
    """m, k, g of n cells by 2-point Gauss-Legendre on the pieces between cell
    centres (the tents are linear there), with each tent mirrored across both
    outer faces: evenly for scalars, oddly for a normal vector component."""
    L = n * h
    c = (np.arange(n) + 0.5) * h
    brk = np.concatenate([[0.0], c, [L]])
    gx, gw = np.polynomial.legendre.leggauss(2)
    xs, ws = [], []
    for a, b in zip(brk[:-1], brk[1:]):
        xs.append(0.5 * (b - a) * gx + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * gw)
    x, w = np.concatenate(xs), np.concatenate(ws)
    even = lambda p: _tent(x, c[p], h) + _tent(x, -c[p], h) + _tent(x, 2 * L - c[p], h)
    deven = lambda p: _dtent(x, c[p], h) + _dtent(x, -c[p], h) + _dtent(x, 2 * L - c[p], h)
    odd = lambda p: _tent(x, c[p], h) - _tent(x, -c[p], h) - _tent(x, 2 * L - c[p], h)
    m = np.array([[np.sum(w * even(p) * even(q)) / h for q in range(n)] for p in range(n)])
    k = np.array([[np.sum(w * deven(p) * deven(q)) * h for q in range(n)] for p in range(n)])
    g = np.array([[np.sum(w * deven(p) * odd(q)) for q in range(n)] for p in range(n)])
    return m, k, g


@pytest.mark.parametrize("n", [2, 3, 6])
def test_one_dimensional_matrices_by_quadrature(n):
    m, k, g = _quad_1d(n)
    assert np.allclose(G.mass_1d(n), m, atol=1e-14)
    assert np.allclose(G.stiff_1d(n), k, atol=1e-14)
    assert np.allclose(G.deriv_1d(n), g, atol=1e-14)


def test_interior_stencil_is_the_27_point_q1_stiffness():
    # h {8/3, 0, -1/6, -1/12} (centre, face, edge, corner neighbours) in units of h
    e = np.zeros((5, 5, 5))
    e[2, 2, 2] = 1.0
    col = G.apply_A(e)
    assert col[2, 2, 2] == pytest.approx(8.0 / 3.0)
    assert col[2, 2, 3] == pytest.approx(0.0, abs=1e-15)
    assert col[2, 3, 3] == pytest.approx(-1.0 / 6.0)
    assert col[3, 3, 3] == pytest.approx(-1.0 / 12.0)
    assert abs(col.sum()) < 1e-14


def test_boundary_rows_are_the_stencil_with_clamped_indices():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 5, 6))
    coef = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}
    want = np.zeros_like(x)
    nz, ny, nx = x.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            kk, jj, ii = (min(max(k + dz, 0), nz - 1), min(max(j + dy, 0), ny - 1),
                                          min(max(i + dx, 0), nx - 1))
                            want[k, j, i] += coef[abs(dx) + abs(dy) + abs(dz)] * x[kk, jj, ii]
    assert np.allclose(G.apply_A(x), want, atol=1e-13)


def test_lumped_mass_gives_the_vertex_quadrature_system(monkeypatch):
    grid = D.Grid((6, 5, 4), (0.1, 0.2, 0.3), 0.125)
    rng = np.random.default_rng(6)
    V = rng.standard_normal((3,) + grid.shape)
    chi = rng.standard_normal(grid.shape)
    monkeypatch.setattr(G, "mass_1d", lambda n: np.eye(n))
    assert np.allclose(G.divergence(grid, V), D.divergence(grid, V), atol=1e-13)
    assert np.allclose(G.apply_A(chi), D.apply_A(chi), atol=1e-13)


def test_cosine_modes_are_eigenvectors():
    shape = (5, 6, 7)
    lam = G.eigenvalues(shape)
    for q in [(0, 0, 1), (2, 3, 1), (4, 5, 6)]:
        idx = np.indices(shape)
        u = np.ones(shape)
        for ax in range(3):
            u = u * np.cos(np.pi * q[ax] * (idx[ax] + 0.5) / shape[ax])
        assert np.allclose(G.apply_A(u), lam[q] * u, atol=1e-12)


def test_dct_solve_equals_dense_conjugate_gradients():
    shape = (4, 5, 6)
    N = int(np.prod(shape))
    Amat = np.stack([G.apply_A(e.reshape(shape)).ravel() for e in np.eye(N)], axis=1)
    b = np.random.default_rng(7).standard_normal(N)
    b -= b.mean()
    x = np.zeros(N)
    r = b - Amat @ x
    p = r.copy()
    for _ in range(4 * N):
        Ap = Amat @ p
        a = (r @ r) / (p @ Ap)
        x += a * p
        rn = r - a * Ap
        if np.linalg.norm(rn) < 1e-14 * np.linalg.norm(b):
            r = rn
            break
        p = rn + (rn @ rn) / (r @ r) * p
        r = rn
    x -= x.mean()
    assert np.allclose(G.solve(b.reshape(shape)).ravel(), x, atol=1e-11)


def test_divergence_transpose():
    grid = D.Grid((5, 6, 4), (0.0, 0.0, 0.0), 0.2)
    rng = np.random.default_rng(8)
    V = rng.standard_normal((3,) + grid.shape)
    lam = rng.standard_normal(grid.shape)
    lhs = np.sum(G.divergence(grid, V) * lam)
    rhs = np.sum(V * G.divergence_T(grid, lam))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
