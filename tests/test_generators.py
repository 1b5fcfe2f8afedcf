"""Invariants of the seeded synthetic workloads (inputs only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from shapley_inputs import configs, games
from shapley_inputs.games import Grid


def row_sums(g):
    return np.add.reduceat(np.r_[g.w, 0.0], g.row_ptr[:-1]) * (np.diff(g.row_ptr) > 0)


@pytest.mark.parametrize("make", [lambda: configs.c0(), lambda: configs.c1(points=65),
                                  lambda: configs.c2(s=9), lambda: configs.c3_game(3, 17, 0.5),
                                  lambda: configs.c4_game(1, 40, 2.0, 2001),
                                  lambda: games.two_stopper_game(33)])
def test_stencil_games_are_substochastic(make):
    g = make()
    g.check()
    s = row_sums(g)
    assert np.all(s <= 1.0 + 1e-15)
    # every policy system I - W^{ab} is a (weakly) diagonally dominant M-matrix
    W = sp.csr_matrix((g.w, g.col, g.row_ptr), shape=(g.nrows, g.n))
    assert W.min() >= 0


def test_config_sizes_match_the_recipes():
    g = configs.c0()
    assert (g.n, g.m1, g.m2, g.nrows, g.nnz) == (1089, 3, 3, 9801, 38016)
    g = configs.c1(points=129)
    assert (g.n, g.m1, g.m2) == (127 ** 2, 2, 1)
    # stop rows are empty, continuation rows have the 5-point stencil minus the diagonal
    lens = np.diff(g.row_ptr).reshape(g.n, 2)
    assert np.all(lens[:, 0] == 0) and lens[:, 1].max() == 4
    g = configs.c2(s=9)
    assert (g.n, g.m1, g.m2) == (729, 3, 3)
    assert np.diff(g.row_ptr).max() == 6


def test_normalised_upwind_weights():
    """q_{+-k} = 0.5 + h d_k^{+-}, D = dim + h sum|d| + h^2 lambda (Sec. 3.3)."""
    s, lam = 7, 2.0
    grid = Grid(2, s)
    g = games.isaacs_game(grid, np.zeros(grid.n), lam)
    h = grid.h
    x = 3 + s * 3  # an interior state away from the boundary
    for a in range(3):
        for b in range(3):
            i = (x * 3 + a) * 3 + b
            cols = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
            w = g.w[g.row_ptr[i]:g.row_ptr[i + 1]]
            d1, d2 = a - 1.0, b - 1.0
            D = 2 + h * (abs(d1) + abs(d2)) + h * h * lam
            expect = {x - s: (0.5 + h * max(-d2, 0)) / D, x - 1: (0.5 + h * max(-d1, 0)) / D,
                      x + 1: (0.5 + h * max(d1, 0)) / D, x + s: (0.5 + h * max(d2, 0)) / D}
            assert dict(zip(cols.tolist(), w.tolist())) == pytest.approx(expect, rel=1e-15)
            r = -0.1 * d1 ** 2 + 0.1 * d2 ** 2
            assert g.r[i] == pytest.approx(h * h * r / D, rel=1e-14, abs=1e-18)


def test_obstacle_recipe_has_a_free_boundary():
    g = configs.c1(points=65)
    import oracle
    res = oracle.policy_iteration(g)
    assert 0.2 <= np.mean(res.alpha == 0) <= 0.8


def test_c3_and_c4_distributions():
    side, lam = configs.c3_sizes()
    assert len(side) == 256 and set(np.unique(side)) <= {65, 129, 257}
    assert lam.min() >= 0.1 and lam.max() <= 10.0
    assert abs(np.mean(side ** 2) * 256 / 7.42e6 - 1) < 0.1
    req = configs.c4_requests()
    kinds = np.array([r[0] for r in req])
    sides = np.array([r[1] for r in req])
    assert 0.4 < kinds.mean() < 0.6
    assert sides.min() >= 33 and sides.max() <= 1025
    med = np.median(sides ** 2)
    assert 2.0e4 < med < 5.0e4


def test_nested_levels():
    levels = configs.c1_levels(points=129, coarsest_points=17)
    assert [g.meta["points"] for g in levels] == [17, 33, 65, 129]
    hs = [1.0 / (g.grid.s + 1) for g in levels]
    assert all(abs(hs[i] / hs[i + 1] - 2.0) < 1e-12 for i in range(len(hs) - 1))
