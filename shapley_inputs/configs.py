"""Seeded recipes of the five benchmark workloads (inputs only).

C0  Isaacs 2-D, 33x33 interior grid, lambda = 1, f = sin(2 pi x1) cos(2 pi x2)
    + 0.1 N(0,1) (seed 0), a, b in {-1,0,1}, d = (a, b).
C1  Obstacle problem on 1025x1025 points (incl. boundary: s = 1023,
    h = 2^-10), lambda = 0.5, f = sum of 8 Gaussian bumps (seed 1) with
    amplitudes U[-25, 25], centres U[0.15, 0.85]^2, widths U[0.04, 0.12]
    (signed amplitudes give a free boundary: about 27% of the states are in
    contact), psi = 0.2 sin(pi x1) sin(pi x2), Dirichlet 0.
C2  Isaacs 3-D on 129^3 interior points, d = (a, b, 0), lambda = 1,
    f = sum of 8 3-D Gaussians (seed 2).
C3  256 Isaacs 2-D games, sides uniform in {65, 129, 257}, lambda
    log-uniform in [0.1, 10], f as in C0 (instance k seeded 1000 + k).
C4  Request stream: 50/50 Isaacs / obstacle, side round(exp U[ln 33,
    ln 1025]), lambda log-uniform in [0.1, 10] (request i seeded 2000 + i).

Every recipe takes its sizes as arguments so that tests can build the same
family at small sizes.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .games import Grid, Game, grid_coords, isaacs_game, obstacle_game


def f_sincos(grid: Grid, rng: np.random.Generator) -> np.ndarray:
    x1, x2 = grid_coords(grid)[:2]
    return np.sin(2 * math.pi * x1) * np.cos(2 * math.pi * x2) + 0.1 * rng.standard_normal(grid.n)


def f_bumps(grid: Grid, rng: np.random.Generator, k: int = 8, amp=(-25.0, 25.0),
            centre=(0.15, 0.85), sigma=(0.04, 0.12)) -> np.ndarray:
    xs = grid_coords(grid)
    A = rng.uniform(*amp, size=k)
    C = rng.uniform(*centre, size=(k, grid.dim))
    S = rng.uniform(*sigma, size=k)
    f = np.zeros(grid.n)
    for j in range(k):
        d2 = sum((xs[t] - C[j, t]) ** 2 for t in range(grid.dim))
        f += A[j] * np.exp(-d2 / (2 * S[j] ** 2))
    return f


def psi_sin(grid: Grid) -> np.ndarray:
    xs = grid_coords(grid)
    out = 0.2 * np.ones(grid.n)
    for t in range(grid.dim):
        out = out * np.sin(math.pi * xs[t])
    return out


def c0(s: int = 33, seed: int = 0, lam: float = 1.0) -> Game:
    grid = Grid(2, s)
    rng = np.random.default_rng(seed)
    g = isaacs_game(grid, f_sincos(grid, rng), lam)
    g.meta.update(config="C0", seed=seed)
    return g


def c1(points: int = 1025, seed: int = 1, lam: float = 0.5) -> Game:
    """`points` per side including the boundary (s = points - 2)."""
    grid = Grid(2, points - 2)
    rng = np.random.default_rng(seed)
    g = obstacle_game(grid, f_bumps(grid, rng), psi_sin(grid), lam)
    g.meta.update(config="C1", seed=seed, points=points)
    return g


def c1_levels(points: int = 1025, coarsest_points: int = 33, seed: int = 1,
              lam: float = 0.5) -> List[Game]:
    """Nested rediscretisations of C1, coarse -> fine, h_l = 2^l h.

    The bump parameters are drawn once (same seed) and sampled on every grid.
    """
    out = []
    p = coarsest_points
    while p <= points:
        out.append(c1(p, seed, lam))
        p = 2 * (p - 1) + 1
    assert out[-1].meta["points"] == points, "points must be 2^k (coarsest-1) + 1"
    return out


def c2(s: int = 129, seed: int = 2, lam: float = 1.0) -> Game:
    grid = Grid(3, s)
    rng = np.random.default_rng(seed)
    f = f_bumps(grid, rng, amp=(-1.0, 1.0), centre=(0.1, 0.9), sigma=(0.05, 0.2))
    g = isaacs_game(grid, f, lam)
    g.meta.update(config="C2", seed=seed)
    return g


def c3_sizes(count: int = 256, master_seed: int = 3, sides=(65, 129, 257)):
    rng = np.random.default_rng(master_seed)
    side = rng.choice(np.asarray(sides), size=count)
    lam = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=count))
    return side.astype(int), lam


def c3_game(k: int, side: int, lam: float) -> Game:
    grid = Grid(2, int(side))
    rng = np.random.default_rng(1000 + k)
    g = isaacs_game(grid, f_sincos(grid, rng), float(lam))
    g.meta.update(config="C3", instance=k)
    return g


def c3(count: int = 256, master_seed: int = 3, sides=(65, 129, 257)) -> List[Game]:
    side, lam = c3_sizes(count, master_seed, sides)
    return [c3_game(k, side[k], lam[k]) for k in range(count)]


def c4_requests(count: int = 1000, master_seed: int = 4, smin: int = 33, smax: int = 1025):
    """(kind, side, lambda, seed) per request; kind 0 Isaacs, 1 obstacle."""
    rng = np.random.default_rng(master_seed)
    kind = rng.integers(0, 2, size=count)
    side = np.rint(np.exp(rng.uniform(math.log(smin), math.log(smax), size=count))).astype(int)
    lam = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=count))
    return [(int(kind[i]), int(side[i]), float(lam[i]), 2000 + i) for i in range(count)]


def c4_game(kind: int, side: int, lam: float, seed: int) -> Game:
    grid = Grid(2, side)
    rng = np.random.default_rng(seed)
    if kind == 0:
        g = isaacs_game(grid, f_sincos(grid, rng), lam)
    else:
        g = obstacle_game(grid, f_bumps(grid, rng), psi_sin(grid), lam)
    g.meta.update(config="C4", seed=seed, kind=kind)
    return g


def obstacle_levels_for_side(side: int, seed: int, lam: float, coarsest_max: int = 32):
    """Non-nested coarse hierarchy for an obstacle request of interior side s.

    Intervals m_l = ceil(m_{l-1} / 2) down to at most `coarsest_max`
    intervals; returned coarse -> fine.  Reduces to the dyadic hierarchy when
    the finest interval count is a power of two.
    """
    m = side + 1
    ms = [m]
    while m > coarsest_max:
        m = (m + 1) // 2
        ms.append(m)
    out = []
    for mm in reversed(ms):
        grid = Grid(2, mm - 1)
        rng = np.random.default_rng(seed)
        out.append(obstacle_game(grid, f_bumps(grid, rng), psi_sin(grid), lam))
    return out
