"""Grids over a cloud's bounding box (paper Sec. 2.3, Table 1's grid density
d): the oracle's reading pinned on a hand-worked case and on invariants, and
the library's host arithmetic (wg_grid_from_bbox) equal to it."""
import numpy as np
import pytest

from oracle import domain


def _levels(n):
    """Extents of a hierarchy that halves every extent while all are even and
    >= 4 and one exceeds 32 (the solver's rule)."""
    out = [tuple(n)]
    while all(v % 2 == 0 and v >= 4 for v in out[-1]) and max(out[-1]) > 32:
        out.append(tuple(v // 2 for v in out[-1]))
    return out


def test_hand_worked_box():
    # h = 1/256; the box 208 x 72 x 96 cells, widened by 3 per side: 214, 78, 102.
    # 214 / 2^3 <= 32 -> q = 8: 216, 80, 104; centred at the box centre.
    g = domain.grid_over_box((0.25, 0.375, 0.5), (1.0625, 0.65625, 0.875), 256.0, pad=3)
    assert g.n == (216, 80, 104) and g.h == 1.0 / 256
    assert g.lo == (0.234375, 0.359375, 0.484375)


@pytest.mark.parametrize("seed", range(6))
def test_invariants_on_random_boxes(seed):
    rng = np.random.default_rng(900 + seed)
    lo = rng.uniform(-1, 1, 3)
    hi = lo + rng.uniform(0.01, 1.5, 3) * rng.choice([0.05, 1.0], 3)
    d = float(rng.uniform(20, 300))
    pad = int(rng.integers(0, 5))
    g = domain.grid_over_box(lo, hi, d, pad)
    n, glo, h = np.array(g.n), np.array(g.lo), g.h
    # the box with its pad lies inside the grid (to rounding)
    assert np.all(glo <= lo - pad * h + 1e-9) and np.all(glo + n * h >= hi + pad * h - 1e-9)
    # the hierarchy ends at <= 32 cells per axis
    assert max(_levels(n)[-1]) <= 32
    # minimal: one step of q less would not cover the padded box or fall below 2q
    L = len(_levels(n)) - 1
    q = 2 ** L
    need = np.maximum(np.ceil((hi - lo) / h) + 2 * pad, 1)
    assert np.all(n % q == 0) and np.all((n - q < need) | (n == 2 * q))
    # centred
    assert np.allclose(glo + n * h / 2, (lo + hi) / 2)


@pytest.mark.parametrize("seed", range(6))
def test_library_grid_equals_oracle(seed):
    from paper_2609_20964_amd import _lib
    rng = np.random.default_rng(950 + seed)
    lo = rng.uniform(-1, 1, 3)
    hi = lo + rng.uniform(0.01, 1.5, 3)
    d, pad = float(rng.uniform(20, 300)), int(rng.integers(0, 5))
    g = domain.grid_over_box(lo, hi, d, pad)
    n, glo, h = _lib.grid_from_bbox(lo, hi, d, pad)
    assert n == g.n and h == g.h and glo == g.lo


def test_library_rejects_bad_boxes():
    from paper_2609_20964_amd import _lib
    with pytest.raises(_lib.WgError):
        _lib.grid_from_bbox((0, 0, 0), (1, 1, 1), 0.0)
    with pytest.raises(_lib.WgError):
        _lib.grid_from_bbox((0, 0, 0), (1, -1, 1), 10.0)
