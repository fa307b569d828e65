"""Pins of the surrogate's fallback and out-of-distribution oracles (CPU).

The fallback rebuilds a cell's particles from its moments at the quantiles
of a lognormal: the rebuilt set must carry the cell's M0 to the rounding of
the multiplicity and M1 and M2 exactly (up to rounding) beyond it; with
M2 M0 = M1^2 (a monodisperse cell) every volume is the mean volume.  The occupancy test is checked on hand-built
inputs."""
import math

import numpy as np

from oracle import mlp


def _moments(xi, v, dv):
    xi = xi.astype(np.float64)
    return np.array([xi.sum(), (xi * v).sum(), (xi * v * v).sum()]) / dv


def test_seeded_cell_reproduces_its_moments():
    dv = 2500.0
    # a lognormal cell: N0 = 1e8 m^-3, median radius 10 um, sigma_g 1.5
    s2 = (3.0 * math.log(1.5)) ** 2
    mu = math.log(4.0 / 3.0 * math.pi * 1e-5 ** 3)
    N0 = 1e8
    M = np.array([[N0, N0 * math.exp(mu + s2 / 2), N0 * math.exp(2 * mu + 2 * s2)]])
    for n in (64, 512, 4096):
        xi, v = mlp.seed_from_moments(M, None, n, dv)
        got = _moments(xi, v, dv)
        e0 = got[0] / M[0, 0] - 1
        assert abs(e0) <= 0.5 * n / (N0 * dv) + 1e-15          # multiplicity rounding
        assert abs((got[1] / M[0, 1] - 1) - e0) < 1e-12
        assert abs((got[2] / M[0, 2] - 1) - e0) < 1e-12
        # the spread is the lognormal's, not a two-point set: quantiles of
        # one distribution, sorted, from below to above the mean volume
        assert np.all(np.diff(v) > 0) and v[0] < M[0, 1] / M[0, 0] < v[-1]


def test_seeded_ratio_beyond_reach_is_capped():
    """n SDs of one multiplicity hold at most n times the squared mean: a
    larger M2 M0 / M1^2 saturates (M1 still exact)."""
    n = 8
    xi, v = mlp.seed_from_moments(np.array([[8e6, 8e6, 8e12]]), None, n, 1.0)
    got = _moments(xi, v, 1.0)
    ratio = got[2] * got[0] / got[1] ** 2
    assert abs(got[1] / 8e6 - 1) < 1e-12 and 0.9 * n < ratio <= n * (1 + 1e-12)


def test_monodisperse_cell_and_unselected_cells():
    dv = 1e6
    M = np.array([[2.0, 6.0, 18.0], [1.0, 1.0, 5.0], [0.0, 0.0, 0.0]])  # cell 0: v = 3
    xi, v = mlp.seed_from_moments(M, np.array([1, 0, 1], np.uint8), 8, dv)
    assert np.all(v[:8] == 3.0) and np.all(xi[:8] == np.uint64(250000))
    assert np.all(xi[8:] == 0) and np.all(v[8:] == 0)        # unselected, empty


def test_multiplicity_is_at_least_one():
    xi, v = mlp.seed_from_moments(np.array([[1e-9, 1e-20, 1e-30]]), None, 16, 1.0)
    assert np.all(xi == 1)


def test_occupancy_test_by_hand():
    lo = np.array([0, 0, 0, -1, -1], np.float32)
    hi = np.array([4, 4, 4, 1, 1], np.float32)
    train = np.array([[0.5, 0.5, 0.5, 0, 0], [3.9, 3.9, 3.9, 0, 0], [2.0, 1.0, 3.0, 0, 0]],
                     np.float32)
    occ, glo, ginv = mlp.occupancy(train, lo, hi, 4)
    assert occ.sum() == 3 and occ[0, 0, 0] and occ[3, 3, 3] and occ[2, 1, 3]
    x = np.array([[0.1, 0.9, 0.2, 0, 0],    # cell (0,0,0): inside
                  [2.5, 1.5, 3.5, 0, 0],    # cell (2,1,3): inside
                  [1.5, 1.5, 1.5, 0, 0],    # empty cell, inside the box
                  [4.0, 4.0, 4.0, 0, 0],    # the box's upper corner: cell (3,3,3)
                  [0.5, 0.5, 0.5, 2, 0],    # outside the box in feature 3
                  [np.nan, 0.5, 0.5, 0, 0]], np.float32)
    assert list(mlp.ood_fallback(x, lo, hi, occ, glo, ginv)) == [0, 0, 1, 0, 1, 1]
    assert list(mlp.ood_fallback(x, lo, hi)) == [0, 0, 0, 0, 1, 1]   # box only


def test_merge():
    M = np.arange(9, dtype=np.float64).reshape(3, 3)
    S = -M
    out = mlp.moments_merge(M, S, np.array([0, 1, 0], np.uint8))
    assert np.array_equal(out, np.array([[0, 1, 2], [-3, -4, -5], [6, 7, 8]], np.float64))
