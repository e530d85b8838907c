"""Pins of the numpy V-cycle that the GPU preconditioner is compared with:
M is symmetric, the stationary iteration x <- x + M (b - A x) contracts the
residual by well over 5x per step (so M approximates A^-1; a wrong sign,
weight or transfer breaks this), P reproduces constants under zero flux, and
a single-level hierarchy is the exact solve."""
import numpy as np
import pytest

import mg_reference as MG
from oracle import discretize as D


@pytest.mark.parametrize("shape,bc", [((24, 40, 48), "neumann"), ((20, 20, 36), "dirichlet"),
                                      ((36, 40, 66), "neumann")])
def test_symmetric(shape, bc):
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(shape), rng.standard_normal(shape)
    lhs, rhs = np.vdot(MG.apply(a, bc), b), np.vdot(a, MG.apply(b, bc))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("shape,bc", [((64, 64, 64), "neumann"), ((24, 40, 48), "dirichlet")])
def test_stationary_iteration_contracts(shape, bc):
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


def test_single_level_is_exact():
    rng = np.random.default_rng(5)
    b = rng.standard_normal((16, 12, 10))
    b -= b.mean()
    x = MG.apply(b, "neumann")
    assert np.linalg.norm(D.apply_A(x, "neumann") - b) <= 1e-10 * np.linalg.norm(b)
