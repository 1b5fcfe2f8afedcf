"""Seeded synthetic game builders shared by the oracle and the GPU path.

This module only *builds inputs*: it turns a PDE, a grid and seeded random
coefficients into the finite game of the Shapley equation
    v(x) = max_a min_b ( sum_y mu p(y|x,a,b) v(y) + r(x,a,b) )
(Akian & Detournay, Sec. 2, eq. (eq1)).  It solves nothing: no value,
policy or linear-system arithmetic of the method lives here.

Game layout (one CSR row per triple (x, a, b), b fastest):
    row(x, a, b) = (x * m1 + a) * m2 + b
    row_ptr[int64, n*m1*m2+1], col[int32], w[float64] = mu_ab * p(y|x,a,b),
    r[float64] = normalised running reward (boundary terms folded in),
    mu = 1.0 (the action-dependent discount is folded into w, see below),
    valid[uint8, n*m1*m2] or None.

Finite-difference discretisation (Sec. 3.3, schemes (decent) and (centre);
the normalisation follows the worked example (Iex1d), Sec. 6.1): for a
drift d(a,b) and diffusion 0.5*I in dimension `dim`, at grid step h,
    q_{+k} = 0.5 + h max(d_k, 0),  q_{-k} = 0.5 + h max(-d_k, 0),
    c = sum q = dim + h sum_k |d_k|,   D = c + h^2 lambda,
    w(x -> y) = q_y / D for interior neighbours y,
    r~ = h^2 r(x,a,b) / D + sum over boundary neighbours y of q_y/D g(y).
The discount mu_ab = c/D < 1 is folded into w, so mu = 1 is passed.

States are numbered x = (i-1) + s (j-1) [+ s^2 (k-1)], x1 fastest, with s
interior points per side and h = 1/(s+1).  Action indices ascend by value:
{-1, 0, 1} -> {0, 1, 2}; for stopping games stop = 0, continue = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Grid:
    """Uniform grid on the unit cube: `s` interior points per side."""
    dim: int
    s: int
    periodic: bool = False
    # values of the Dirichlet data on the extended (s+2)^dim grid, x1 fastest;
    # only boundary nodes are meaningful.  None means g = 0.
    bvals: Optional[np.ndarray] = None

    @property
    def h(self) -> float:
        return 1.0 / (self.s if self.periodic else self.s + 1)

    @property
    def n(self) -> int:
        return self.s ** self.dim


@dataclasses.dataclass
class Game:
    n: int
    m1: int
    m2: int
    row_ptr: np.ndarray   # int64 [n*m1*m2 + 1]
    col: np.ndarray       # int32 [nnz]
    w: np.ndarray         # float64 [nnz]
    r: np.ndarray         # float64 [n*m1*m2]
    mu: float = 1.0
    valid: Optional[np.ndarray] = None   # uint8 [n*m1*m2]
    grid: Optional[Grid] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nrows(self) -> int:
        return self.n * self.m1 * self.m2

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def nbytes(self) -> int:
        b = self.row_ptr.nbytes + self.col.nbytes + self.w.nbytes + self.r.nbytes
        return b + (self.valid.nbytes if self.valid is not None else 0)

    def check(self) -> None:
        """Structural sanity of the CSR arrays (not of the method)."""
        nr = self.nrows
        assert self.row_ptr.dtype == np.int64 and self.row_ptr.shape == (nr + 1,)
        assert self.row_ptr[0] == 0 and np.all(np.diff(self.row_ptr) >= 0)
        assert self.col.dtype == np.int32 and self.col.shape == (self.nnz,)
        assert self.w.dtype == np.float64 and self.w.shape == (self.nnz,)
        assert self.r.dtype == np.float64 and self.r.shape == (nr,)
        if self.nnz:
            assert self.col.min() >= 0 and self.col.max() < self.n
        assert np.all(self.w >= 0)


# ----------------------------------------------------------------------------
# grid helpers
# ----------------------------------------------------------------------------

def grid_coords(grid: Grid):
    """Coordinates of interior nodes, each an array of shape (n,), x1 fastest."""
    h = grid.h
    idx = np.arange(1, grid.s + 1) * h if not grid.periodic else np.arange(grid.s) * h
    mesh = np.meshgrid(*([idx] * grid.dim), indexing="ij")
    # meshgrid 'ij' makes the first axis slowest; flip so x1 is fastest
    return [m.transpose(tuple(range(grid.dim))[::-1]).reshape(-1) for m in mesh]


def _bval_lookup(grid: Grid, ext_index: np.ndarray) -> np.ndarray:
    if grid.bvals is None:
        return np.zeros(ext_index.shape, dtype=np.float64)
    return grid.bvals[ext_index]


def _stencil_rows(grid: Grid, drifts: np.ndarray, lam: np.ndarray, reward: np.ndarray):
    """Rows of the normalised upwind scheme for all (x, action) pairs.

    drifts: (n, K, dim) drift per state and action pair; lam: (n, K) or scalar
    broadcastable; reward: (n, K) running reward r(x, action).
    Returns (cols (n,K,2dim) int64 with -1 for boundary, w (n,K,2dim), rt (n,K)).
    """
    dim, s, h = grid.dim, grid.s, grid.h
    n = grid.n
    K = drifts.shape[1]
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (n, K))
    # multi-index of each state, 0-based interior index per axis
    x = np.arange(n)
    sub = [(x // s ** k) % s for k in range(dim)]
    q = np.empty((n, K, 2 * dim))
    cols = np.empty((n, K, 2 * dim), dtype=np.int64)
    bidx = np.zeros((n, 2 * dim), dtype=np.int64)   # extended-grid index of boundary nbr
    for k in range(dim):
        dk = drifts[:, :, k]
        q[:, :, 2 * k] = 0.5 + h * np.maximum(-dk, 0.0)      # neighbour x - h e_k
        q[:, :, 2 * k + 1] = 0.5 + h * np.maximum(dk, 0.0)   # neighbour x + h e_k
        for side, step in ((0, -1), (1, +1)):
            nb = sub[k] + step
            if grid.periodic:
                nb = nb % s
                lin = x + (nb - sub[k]) * s ** k
                cols[:, :, 2 * k + side] = lin[:, None]
            else:
                inside = (nb >= 0) & (nb < s)
                lin = np.where(inside, x + step * s ** k, -1)
                cols[:, :, 2 * k + side] = lin[:, None]
                # extended-grid index (coordinates shifted by one)
                ext = np.zeros(n, dtype=np.int64)
                for kk in range(dim):
                    c = sub[kk] + 1 + (step if kk == k else 0)
                    ext += c * (s + 2) ** kk
                bidx[:, 2 * k + side] = np.where(inside, -1, ext)
    c = q.sum(axis=2)
    D = c + h * h * lam
    w = q / D[:, :, None]
    rt = h * h * reward / D
    if not grid.periodic:
        bmask = cols < 0
        if bmask.any():
            gvals = np.zeros((n, 2 * dim))
            sel = bidx >= 0
            gvals[sel] = _bval_lookup(grid, bidx[sel])
            rt = rt + np.where(bmask, w * gvals[:, None, :], 0.0).sum(axis=2)
    return cols, w, rt


def _assemble(n: int, m1: int, m2: int, cols: np.ndarray, w: np.ndarray,
              rt: np.ndarray, empty_rows: Optional[np.ndarray] = None) -> tuple:
    """Pack (n, m1*m2, slots) stencil rows into CSR with ascending columns.

    Slots with col < 0 (boundary) are dropped.  `empty_rows` (n, m1*m2) bool
    marks rows that carry no transition at all (e.g. a stopping action).
    """
    K = m1 * m2
    cols = cols.reshape(n * K, -1)
    w = w.reshape(n * K, -1)
    keep = cols >= 0
    if empty_rows is not None:
        keep &= ~empty_rows.reshape(n * K, 1)
    order = np.argsort(np.where(keep, cols, np.iinfo(np.int64).max), axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    w = np.take_along_axis(w, order, axis=1)
    keep = np.take_along_axis(keep, order, axis=1)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(n * K + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[keep].astype(np.int32)
    wv = w[keep].astype(np.float64)
    return row_ptr, col, wv, rt.reshape(n * K).astype(np.float64)


# ----------------------------------------------------------------------------
# Isaacs games (Sec. 3.1, eq. (BIcont1); example (Iex1)/(Iex1d) in Sec. 6.1)
# ----------------------------------------------------------------------------

ACTIONS_3 = np.array([-1.0, 0.0, 1.0])


def isaacs_game(grid: Grid, f: np.ndarray, lam: float,
                a_vals: Sequence[float] = ACTIONS_3, b_vals: Sequence[float] = ACTIONS_3,
                drift: Optional[Callable] = None,
                reward: Optional[Callable] = None) -> Game:
    """max_a min_b (0.5 Lap v + d(a,b).grad v - lam v + r(x,a,b)) = 0.

    Defaults follow the benchmark recipe: d = (a, b, 0, ...) and
    r(x,a,b) = f(x) - 0.1 a^2 + 0.1 b^2.
    """
    a_vals = np.asarray(a_vals, dtype=np.float64)
    b_vals = np.asarray(b_vals, dtype=np.float64)
    m1, m2 = len(a_vals), len(b_vals)
    n, dim = grid.n, grid.dim
    A, B = np.meshgrid(a_vals, b_vals, indexing="ij")      # (m1, m2), b fastest
    A = A.reshape(-1)
    B = B.reshape(-1)
    K = m1 * m2
    if drift is None:
        d = np.zeros((K, dim))
        d[:, 0] = A
        if dim > 1:
            d[:, 1] = B
        drifts = np.broadcast_to(d, (n, K, dim))
    else:
        drifts = drift(A, B)
    if reward is None:
        rew = f[:, None] - 0.1 * A[None, :] ** 2 + 0.1 * B[None, :] ** 2
    else:
        rew = reward(f, A, B)
    cols, w, rt = _stencil_rows(grid, np.ascontiguousarray(drifts), lam, rew)
    row_ptr, col, wv, r = _assemble(n, m1, m2, cols, w, rt)
    g = Game(n, m1, m2, row_ptr, col, wv, r, 1.0, None, grid,
             meta=dict(kind="isaacs", lam=lam))
    return g


def obstacle_game(grid: Grid, f: np.ndarray, psi: np.ndarray, lam: float) -> Game:
    """Stopping game (Sec. 3.2, eq. (VI)): v = max(psi, cont(v)), MAX may stop.

    a = 0 (stop): empty row, r~ = psi(x); a = 1 (continue): the normalised
    0.5 Lap - lam scheme with r~ = h^2 f / D.  m2 = 1 (no MIN action).
    """
    n, dim = grid.n, grid.dim
    K = 2
    drifts = np.zeros((n, K, dim))
    rew = np.stack([np.zeros(n), f], axis=1)
    cols, w, rt = _stencil_rows(grid, drifts, lam, rew)
    rt[:, 0] = psi
    empty = np.zeros((n, K), dtype=bool)
    empty[:, 0] = True
    row_ptr, col, wv, r = _assemble(n, 2, 1, cols, w, rt, empty)
    return Game(n, 2, 1, row_ptr, col, wv, r, 1.0, None, grid,
                meta=dict(kind="obstacle", lam=lam))


# ----------------------------------------------------------------------------
# 1-D games
# ----------------------------------------------------------------------------

def dirichlet_1d_game(s: int, r0: float, g0: float = 0.0, g1: float = 0.0) -> Game:
    """One-action game for 0.5 v'' = -r0 on (0,1), v(0)=g0, v(1)=g1, lam = 0."""
    bv = np.zeros(s + 2)
    bv[0], bv[-1] = g0, g1
    grid = Grid(1, s, bvals=bv)
    n = s
    cols, w, rt = _stencil_rows(grid, np.zeros((n, 1, 1)), 0.0, np.full((n, 1), r0))
    row_ptr, col, wv, r = _assemble(n, 1, 1, cols, w, rt)
    return Game(n, 1, 1, row_ptr, col, wv, r, 1.0, None, grid, meta=dict(kind="dirichlet1d"))


def two_stopper_psi_bar() -> float:
    """Obstacle level of the two-stopper example (Sec. 6.3, eq. (exVI2stop))."""
    return (2.0 * math.cos(0.09 * math.pi) + math.pi * (0.18 - 1.0) * math.sin(0.09 * math.pi)) / 2.0


def two_stopper_exact(x: np.ndarray) -> np.ndarray:
    """Closed-form viscosity solution of the two-stopper example (Sec. 6.3)."""
    pb = two_stopper_psi_bar()
    c = pb - math.cos(0.09 * math.pi) - 0.09 * math.pi * math.sin(0.09 * math.pi)
    mid = np.cos(math.pi * x) + math.pi * math.sin(0.09 * math.pi) * x + c
    return np.where(x < 0.09, pb, np.where(x > 0.91, -pb, mid))


def two_stopper_game(points: int) -> Game:
    """1-D two-stopper game on [0,1] with `points` grid points incl. boundary.

    max{psi1 - v, min{psi2 - v, 0.5 v'' + r}} = 0, psi1 = -pb, psi2 = pb,
    r(x) = 0.5 pi^2 cos(pi x) (Sec. 6.3).  Actions: a in {0 stop, 1 continue}
    for MAX, b in {0 stop, 1 continue} for MIN.  Rows (x,0,b) pay psi1;
    (x,1,0) pays psi2; (x,1,1) is the continuation scheme.  Dirichlet data are
    the closed-form values at 0 and 1 (the paper leaves them unstated).
    """
    s = points - 2
    pb = two_stopper_psi_bar()
    bv = np.zeros(s + 2)
    bv[0], bv[-1] = two_stopper_exact(np.array([0.0, 1.0]))
    grid = Grid(1, s, bvals=bv)
    n = s
    (x1,) = grid_coords(grid)
    rx = 0.5 * math.pi ** 2 * np.cos(math.pi * x1)
    K = 4
    drifts = np.zeros((n, K, 1))
    rew = np.zeros((n, K))
    rew[:, 3] = rx
    cols, w, rt = _stencil_rows(grid, drifts, 0.0, rew)
    rt[:, 0] = -pb
    rt[:, 1] = -pb
    rt[:, 2] = pb
    empty = np.zeros((n, K), dtype=bool)
    empty[:, :3] = True
    row_ptr, col, wv, r = _assemble(n, 2, 2, cols, w, rt, empty)
    return Game(n, 2, 2, row_ptr, col, wv, r, 1.0, None, grid, meta=dict(kind="two_stopper"))


# ----------------------------------------------------------------------------
# small random games (for brute-force pins)
# ----------------------------------------------------------------------------

def random_game(n: int, m1: int, m2: int, seed: int, mu: float = 0.9,
                density: float = 0.6, stochastic: bool = False,
                invalid_frac: float = 0.0) -> Game:
    """Random finite game with sparse (sub)stochastic transitions."""
    rng = np.random.default_rng(seed)
    nr = n * m1 * m2
    rows_cols, rows_w = [], []
    for _ in range(nr):
        mask = rng.random(n) < density
        if not mask.any():
            mask[rng.integers(n)] = True
        cols = np.nonzero(mask)[0]
        p = rng.random(len(cols)) + 0.05
        p = p / p.sum()
        if not stochastic:
            p = p * rng.uniform(0.5, 1.0)
        rows_cols.append(cols.astype(np.int32))
        rows_w.append(p)
    counts = np.array([len(c) for c in rows_cols])
    row_ptr = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.concatenate(rows_cols).astype(np.int32)
    w = np.concatenate(rows_w).astype(np.float64)
    r = rng.normal(size=nr)
    valid = None
    if invalid_frac > 0:
        valid = (rng.random(nr) >= invalid_frac).astype(np.uint8).reshape(n, m1, m2)
        # keep at least one valid b for every (x, a)
        for x in range(n):
            for a in range(m1):
                if not valid[x, a].any():
                    valid[x, a, rng.integers(m2)] = 1
        valid = valid.reshape(-1)
    return Game(n, m1, m2, row_ptr, col, w, r, mu, valid, None, meta=dict(kind="random"))


def scale_rows_to_stochastic(g: Game) -> Game:
    """Copy of `g` whose rows sum to one (for the constant-reward closed form)."""
    w = g.w.copy()
    for i in range(g.nrows):
        a, b = g.row_ptr[i], g.row_ptr[i + 1]
        w[a:b] /= w[a:b].sum()
    return dataclasses.replace(g, w=w)


def with_copied_action(g: Game, player: int, src: int, pos: int, dr: float = 0.0) -> Game:
    """Copy of `g` with one more action for `player` (1 = MAX, 2 = MIN),
    inserted at index `pos`, whose rows repeat those of action `src` (indices
    before the insertion) at every state, with `dr` added to their rewards.
    With dr = 0 every state has two actions of identical value: a planted
    exact tie (Sec. 2: argmax and argmin are sets)."""
    m1, m2 = g.m1, g.m2
    m1n, m2n = (m1 + 1, m2) if player == 1 else (m1, m2 + 1)
    src_rows = []  # for each new row (x, a, b): the old row it copies
    for x in range(g.n):
        for a in range(m1n):
            for b in range(m2n):
                if player == 1:
                    ao = src if a == pos else (a if a < pos else a - 1)
                    bo = b
                else:
                    ao = a
                    bo = src if b == pos else (b if b < pos else b - 1)
                src_rows.append(((x * m1 + ao) * m2 + bo, (a == pos) if player == 1 else (b == pos)))
    idx = np.array([s for s, _ in src_rows], dtype=np.int64)
    new = np.array([c for _, c in src_rows], dtype=bool)
    counts = g.row_ptr[idx + 1] - g.row_ptr[idx]
    row_ptr = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    take = np.concatenate([np.arange(g.row_ptr[i], g.row_ptr[i + 1]) for i in idx]).astype(np.int64)
    r = g.r[idx].copy()
    r[new] += dr
    valid = None if g.valid is None else g.valid[idx].copy()
    return Game(g.n, m1n, m2n, row_ptr, g.col[take].copy(), g.w[take].copy(), r, g.mu, valid, g.grid,
                meta=dict(g.meta, copied=(player, src, pos, dr)))


# ----------------------------------------------------------------------------
# games without a grid (the general finite games of Sec. 2)
# ----------------------------------------------------------------------------

def point_cloud_game(n: int, seed: int, k: int = 8, lam: float = 1.0,
                     acts: Sequence[float] = ACTIONS_3, symmetric: bool = True) -> Game:
    """A game on n random points of the unit square whose neighbourhoods are
    those of the symmetric k-nearest-neighbour graph (y is a neighbour of x
    when either is among the other's k nearest; with symmetric=False, x's own
    k nearest only): the upwind weights of the grid scheme with the neighbour
    directions of an unstructured point cloud (no grid, no boundary).

    At x with neighbours y_j (deg of them), unit directions e_j and local step
    hx (the mean neighbour distance), for MAX's action a (drift along x1) and
    MIN's b (drift along x2): q_j = (1 + hx max(0, d . e_j)) / deg with
    d = (a, b), c = sum q_j, D = c + hx^2 lam, w_j = q_j / D, and reward
    r~ = hx^2 (f(x) - 0.1 a^2 + 0.1 b^2) / D with f = sin(2 pi x1) cos(2 pi x2)
    + 0.1 N(0, 1).  The rows are substochastic (sum c/D < 1): mu = 1 is
    passed, as for the grid games."""
    import scipy.sparse as sp
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    _, nbr = cKDTree(pts).query(pts, k=k + 1)
    src = np.repeat(np.arange(n), k)
    dst = nbr[:, 1:].reshape(-1)
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    adj = sp.coo_matrix((np.ones(len(src)), (src, dst)), shape=(n, n)).tocsr()
    adj.setdiag(0)
    adj.eliminate_zeros()
    adj.sort_indices()
    rp, cj = adj.indptr.astype(np.int64), adj.indices.astype(np.int64)
    deg = np.diff(rp)
    xi = np.repeat(np.arange(n), deg)                       # the state of each entry
    dvec = pts[cj] - pts[xi]
    dist = np.hypot(dvec[:, 0], dvec[:, 1])
    e = dvec / np.maximum(dist, 1e-300)[:, None]
    hx = np.add.reduceat(dist, rp[:-1]) / deg
    f = np.sin(2 * np.pi * pts[:, 0]) * np.cos(2 * np.pi * pts[:, 1]) + 0.1 * rng.normal(size=n)
    acts = np.asarray(acts, dtype=np.float64)
    m = len(acts)
    K = m * m
    # rows (x, a, b), b fastest: each repeats the state's neighbour list
    row_len = np.repeat(deg, K)
    row_ptr = np.zeros(n * K + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    col = np.empty(row_ptr[-1], dtype=np.int32)
    w = np.empty(row_ptr[-1])
    r = np.empty(n * K)
    # entry t of state x in row (x, q) sits at row_ptr[x K + q] + t
    t_in = np.arange(len(cj)) - rp[xi]
    for ia, a in enumerate(acts):
        for ib, b in enumerate(acts):
            q = (1.0 + hx[xi] * np.maximum(0.0, a * e[:, 0] + b * e[:, 1])) / deg[xi]
            D = np.add.reduceat(q, rp[:-1]) + hx * hx * lam
            pos = row_ptr[xi * K + ia * m + ib] + t_in
            col[pos] = cj
            w[pos] = q / D[xi]
            r[np.arange(n) * K + ia * m + ib] = hx * hx * (f - 0.1 * a * a + 0.1 * b * b) / D
    return Game(n, m, m, row_ptr, col, w, r, 1.0, None, None,
                meta=dict(kind="point_cloud", k=k, lam=lam, symmetric=symmetric))


def random_sparse_game(n: int, m1: int, m2: int, seed: int, nnz_row: int = 8, mu: float = 0.95,
                       window: Optional[int] = None) -> Game:
    """A random Markov game without geometry: every row (x, a, b) moves to
    nnz_row distinct states drawn uniformly (or, with `window`, from the
    states within `window` of x, cyclically), with random weights summing to
    U[0.5, 1]; normal rewards; discount mu."""
    rng = np.random.default_rng(seed)
    nr = n * m1 * m2
    if window is None:
        cols = rng.integers(0, n, size=(nr, nnz_row))
    else:
        x = np.repeat(np.arange(n), m1 * m2)
        cols = (x[:, None] + rng.integers(-window, window + 1, size=(nr, nnz_row))) % n
    cols = np.sort(cols, axis=1)
    dup = np.zeros_like(cols, dtype=bool)
    dup[:, 1:] = cols[:, 1:] == cols[:, :-1]
    p = rng.random((nr, nnz_row)) + 0.05
    p[dup] = 0.0
    p = p / p.sum(axis=1, keepdims=True) * rng.uniform(0.5, 1.0, size=(nr, 1))
    keep = ~dup
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(nr + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    r = rng.normal(size=nr)
    return Game(n, m1, m2, row_ptr, cols[keep].astype(np.int32), p[keep].astype(np.float64), r, mu, None, None,
                meta=dict(kind="random_sparse", nnz_row=nnz_row, window=window))


# ----------------------------------------------------------------------------
# the Isaacs example with continuous action sets (Sec. 6.1, eqs. (Iex1),
# (Iex1d)), its action sets replaced by finite subsets
# ----------------------------------------------------------------------------

def iex1_exact(x1: np.ndarray, x2: np.ndarray) -> np.ndarray:
    """The exact solution u = sin x1 sin x2 of the example (Sec. 6.1)."""
    return np.sin(x1) * np.sin(x2)


def iex1_game(points: int, a_dirs: int = 8, b_per_axis: int = 5, b_max: float = 1.0,
              lam: float = 0.0) -> Game:
    """Eq. (Iex1) on `points` grid points per direction (boundary included,
    h = 1/(points - 1)), discretised by the upwind scheme as in (Iex1d), with
    the unit disk of MAX replaced by `a_dirs` directions on its boundary circle
    (a linear function of a is maximised on it) and MIN's R^2 by a
    b_per_axis x b_per_axis grid on [0, b_max]^2 (the optimal b = grad u lies
    in [0, 1]^2 on the unit square).  Dirichlet data psi1 = u on the boundary,
    f = -(Lap u + |grad u| - 0.5 |grad u|^2 - lam u).

    (Iex1) carries the full Laplacian; dividing it by two gives the scheme of
    this module with drift (a - b)/2, discount lam/2 and running reward
    (|b|^2/2 + f)/2: the same weights (1 + h (a_k - b_k)^+-)/(c + h^2 lam) and
    rewards h^2 (|b|^2/2 + f)/(c + h^2 lam) as (Iex1d), c = 4 + h|a1 - b1| +
    h|a2 - b2|."""
    s = points - 2
    bv = np.zeros((s + 2, s + 2))
    t = np.arange(s + 2) / (s + 1)
    X1, X2 = np.meshgrid(t, t, indexing="xy")          # x1 fastest in memory
    bv[:, :] = iex1_exact(X1, X2)
    grid = Grid(2, s, bvals=bv.reshape(-1))
    x1, x2 = grid_coords(grid)
    n = grid.n
    gx1, gx2 = np.cos(x1) * np.sin(x2), np.sin(x1) * np.cos(x2)
    gnorm = np.hypot(gx1, gx2)
    f = -(-2.0 * np.sin(x1) * np.sin(x2) + gnorm - 0.5 * gnorm ** 2 - lam * iex1_exact(x1, x2))
    th = 2 * np.pi * np.arange(a_dirs) / a_dirs
    A = np.stack([np.cos(th), np.sin(th)], axis=1)
    bg = np.linspace(0.0, b_max, b_per_axis)
    B = np.array([(u, v) for v in bg for u in bg])
    m1, m2 = len(A), len(B)
    K = m1 * m2
    drifts = np.empty((n, K, 2))
    rew = np.empty((n, K))
    for ia in range(m1):
        for ib in range(m2):
            q = ia * m2 + ib
            drifts[:, q, :] = 0.5 * (A[ia] - B[ib])
            rew[:, q] = 0.5 * (0.5 * (B[ib] @ B[ib]) + f)
    cols, w, rt = _stencil_rows(grid, drifts, 0.5 * lam, rew)
    row_ptr, col, wv, r = _assemble(n, m1, m2, cols, w, rt)
    return Game(n, m1, m2, row_ptr, col, wv, r, 1.0, None, grid,
                meta=dict(kind="iex1", a_dirs=a_dirs, b_per_axis=b_per_axis, b_max=b_max, lam=lam))


def iex1_local_game(points: int, a_dirs: int = 5, b_per_axis: int = 3, da: float = 0.2,
                    db: float = 0.2) -> Game:
    """Eq. (Iex1) discretised as in (Iex1d) with state-dependent finite action
    sets refined around the continuous optimum of the exact solution u
    (a* = grad u / |grad u|, b* = grad u, Sec. 6.1): MAX's directions at angles
    within +-da of a*, MIN's b on a b_per_axis^2 grid within +-db of b*.
    Knowing u, these sets contain the optimum of the discrete operator, so the
    game's value is that of the scheme with exact inner optimisation (a test
    workload: the paper does not state how it optimises over the continuous
    sets).  lam = 0 as in the paper's tests."""
    s = points - 2
    t = np.arange(s + 2) / (s + 1)
    X1, X2 = np.meshgrid(t, t, indexing="xy")
    grid = Grid(2, s, bvals=iex1_exact(X1, X2).reshape(-1))
    x1, x2 = grid_coords(grid)
    n = grid.n
    gx1, gx2 = np.cos(x1) * np.sin(x2), np.sin(x1) * np.cos(x2)
    gn = np.hypot(gx1, gx2)
    f = -(-2.0 * np.sin(x1) * np.sin(x2) + gn - 0.5 * gn ** 2)
    th = np.arctan2(gx2, gx1)[:, None] + np.linspace(-da, da, a_dirs)[None, :]
    A = np.stack([np.cos(th), np.sin(th)], axis=2)                        # (n, m1, 2)
    off = np.linspace(-db, db, b_per_axis)
    B = np.empty((n, b_per_axis * b_per_axis, 2))
    for j, v in enumerate(off):
        for i, u in enumerate(off):
            B[:, j * b_per_axis + i, 0] = gx1 + u
            B[:, j * b_per_axis + i, 1] = gx2 + v
    m1, m2 = a_dirs, b_per_axis * b_per_axis
    drifts = (0.5 * (A[:, :, None, :] - B[:, None, :, :])).reshape(n, m1 * m2, 2)
    rew = np.broadcast_to(0.5 * (0.5 * (B ** 2).sum(axis=2)[:, None, :] + f[:, None, None]), (n, m1, m2))
    cols, w, rt = _stencil_rows(grid, drifts, 0.0, rew.reshape(n, m1 * m2))
    row_ptr, col, wv, r = _assemble(n, m1, m2, cols, w, rt)
    return Game(n, m1, m2, row_ptr, col, wv, r, 1.0, None, grid,
                meta=dict(kind="iex1_local", a_dirs=a_dirs, b_per_axis=b_per_axis, da=da, db=db))
