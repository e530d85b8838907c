"""Pins of the numpy V-cycle that the GPU preconditioner is compared with:
M is symmetric, the stationary iteration x <- x + M (b - A x) contracts the
residual by well over 5x per step (so M approximates A^-1; a wrong sign,
weight or transfer breaks this), P reproduces constants under zero flux, and
a single-level hierarchy (every extent <= 64) is the exact solve.  The shapes
with an extent above 64 have several levels: coarsest solved exactly, or (an
odd coarsest extent above 64) by the Jacobi sweeps."""
import numpy as np
import pytest

import mg_reference as MG
from oracle import discretize as D


@pytest.mark.parametrize("shape,bc", [((24, 40, 80), "neumann"), ((20, 20, 72), "dirichlet"),
                                      ((36, 40, 66), "neumann"), ((130, 8, 8), "neumann")])
def test_symmetric(shape, bc):
    assert len(MG.levels(shape)) > 1
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(shape), rng.standard_normal(shape)
    lhs, rhs = np.vdot(MG.apply(a, bc), b), np.vdot(a, MG.apply(b, bc))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("shape,bc", [((80, 64, 64), "neumann"), ((24, 40, 72), "dirichlet")])
def test_stationary_iteration_contracts(shape, bc):
    assert len(MG.levels(shape)) > 1
    rng = np.random.default_rng(4)
    b = rng.standard_normal(shape)
    if bc == "neumann":
        b -= b.mean()
    x = np.zeros(shape)
    res = [np.linalg.norm(b)]
    for _ in range(4):
        r = b - D.apply_A(x, bc)
        x = x + MG.apply(r, bc)
        r = b - D.apply_A(x, bc)
        if bc == "neumann":
            r -= r.mean()
        res.append(np.linalg.norm(r))
    rates = [res[k + 1] / res[k] for k in range(4)]
    assert max(rates) < 0.2, rates


def test_prolongation_keeps_constants():
    for nf in (8, 10, 34):
        P = MG.prolong_1d(nf, nf // 2, 1)
        assert np.allclose(P.sum(axis=1), 1.0)
        P = MG.prolong_1d(nf, nf // 2, -1)
        assert np.allclose(P.sum(axis=1)[1:-1], 1.0) and np.allclose(P.sum(axis=1)[[0, -1]], 0.5)


@pytest.mark.parametrize("shape", [(16, 12, 10), (64, 48, 40)])
def test_single_level_is_exact(shape):
    assert len(MG.levels(shape)) == 1
    rng = np.random.default_rng(5)
    b = rng.standard_normal(shape)
    b -= b.mean()
    x = MG.apply(b, "neumann")
    assert np.linalg.norm(D.apply_A(x, "neumann") - b) <= 1e-10 * np.linalg.norm(b)


def test_levels():
    assert MG.levels((64, 64, 64)) == [(64, 64, 64)]
    assert MG.levels((66, 40, 36)) == [(66, 40, 36), (33, 20, 18)]
    assert MG.levels((256, 256, 256))[-1] == (32, 32, 32)
    assert MG.levels((130, 8, 8)) == [(130, 8, 8), (65, 4, 4)]
