"""Plain FP64 CPU oracle for the Shapley equation -- TEST INFRASTRUCTURE ONLY.

Only tests, the package's smoke check and the benchmark's CPU-baseline leg may
import this module.  The product path never calls it.

What it computes (Akian & Detournay, arXiv:1107.1653):
  * the dynamic-programming (Shapley) operator
        F(v; x) = max_a min_b ( r(x,a,b) + mu sum_y p(y|x,a,b) v(y) )
    (Sec. 2, eq. (eq1)); its fixed point v* is unique;
  * the value of a pair of pure stationary policies (alpha, beta), i.e. the
    solution of the linear system v = mu M^{alpha beta} v + r^{alpha beta}
    (Sec. 4.2, eq. (LSPI)), here with a sparse direct LU (SciPy SuperLU)
    plus one FP64 refinement step, or -- for 3-D grids of millions of states,
    where the LU fill does not fit in memory -- BiCGSTAB with FP64 residual
    re-checks (a reading; the fixed point is the same);
  * Hoffman-Karp / Puri policy iteration (Sec. 4.2, Algorithm PIalgo) whose
    inner loop is Howard's policy iteration for the MIN player (Sec. 4.1,
    Algorithm algo-MDP), stopped on the residual ||F(v) - v||_inf <= eps
    after each value step (Sec. 5.1) or when no policy improves;
  * the full multilevel scheme FAMGpi (Sec. 5.2, Algorithm algo-FAMGPI) with
    the value interpolation I and the strategy interpolation U.

Readings where the paper is silent (also listed in the design notes):
  * ties: argmax/argmin are sets (Sec. 2).  The incumbent action is kept
    unless another one is better by more than
        tau(x) = 64 * 2^-53 * max over the compared rows of (|r| + mu sum |w||v|),
    the rounding bound of one row evaluation; otherwise the lowest index
    attaining the extremum is taken.
  * the initial MIN policy of an outer step is the argmin at the new alpha
    computed in the same improvement sweep;
  * the inner loop stops when beta is stable; the residual uses the sup-norm;
  * the default start is v0 = 0, alpha0/beta0 greedy at v0.
  * FAMGpi value interpolation I is bi/trilinear on the grid extended by its
    Dirichlet nodes (the paper's neighbour average within distance h_l equals
    it on nested dyadic grids); U copies the coarse node at fine index
    floor(i * (s_c + 1) / (s_f + 1)) clamped to [1, s_c] on each axis.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

TIE_ULPS = 64.0
EPS64 = 2.0 ** -53


@dataclasses.dataclass
class OracleResult:
    v: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    residual: float
    outer: int
    inner_total: int
    log: list
    converged: bool
    seconds: float


def transition_matrix(g) -> sp.csr_matrix:
    """All n*m1*m2 rows of mu-free transition weights as one CSR matrix."""
    return sp.csr_matrix((g.w, g.col.astype(np.int64), g.row_ptr), shape=(g.nrows, g.n))


def _valid(g) -> np.ndarray:
    if g.valid is None:
        return np.ones((g.n, g.m1, g.m2), dtype=bool)
    return g.valid.reshape(g.n, g.m1, g.m2).astype(bool)


def q_values(g, v: np.ndarray, W: Optional[sp.csr_matrix] = None):
    """Q[x,a,b] = r(x,a,b) + mu sum_y w(y|x,a,b) v(y) and its rounding scale.

    Follows the bracket of eq. (eq1) (Sec. 2): one sparse mat-vec over all rows.
    Invalid rows are NaN.
    """
    if W is None:
        W = transition_matrix(g)
    Q = g.r + g.mu * (W @ v)
    absW = abs(W)
    scale = np.abs(g.r) + g.mu * (absW @ np.abs(v))
    Q = Q.reshape(g.n, g.m1, g.m2).copy()
    scale = scale.reshape(g.n, g.m1, g.m2)
    Q[~_valid(g)] = np.nan
    return Q, scale


def _min_over_b(Q):
    return np.nanmin(np.where(np.isnan(Q), np.inf, Q), axis=2)


def shapley_operator(g, v: np.ndarray, W=None) -> np.ndarray:
    """F(v; x) = max_a min_b Q[x,a,b]  (Sec. 2, eq. (eq1))."""
    Q, _ = q_values(g, v, W)
    inner = _min_over_b(Q)                       # +inf if no valid b
    inner = np.where(np.isinf(inner), -np.inf, inner)
    return inner.max(axis=1)


def greedy(g, v: np.ndarray, W=None):
    """Lowest-index argmax_a min_b and argmin_b at that a, with no incumbent."""
    Q, _ = q_values(g, v, W)
    inner = _min_over_b(Q)
    inner_m = np.where(np.isinf(inner), -np.inf, inner)
    alpha = np.argmax(inner_m, axis=1)
    Qa = Q[np.arange(g.n), alpha, :]
    beta = np.argmin(np.where(np.isnan(Qa), np.inf, Qa), axis=1)
    return alpha.astype(np.int32), beta.astype(np.int32)


def policy_system(g, alpha: np.ndarray, beta: np.ndarray, W=None):
    """A = I - mu M^{alpha beta} and b = r^{alpha beta} (Sec. 4.2, eq. (LSPI))."""
    if W is None:
        W = transition_matrix(g)
    sel = (np.arange(g.n) * g.m1 + alpha) * g.m2 + beta
    M = W[sel, :]
    A = (sp.identity(g.n, format="csr") - g.mu * M).tocsr()
    b = g.r[sel].copy()
    return A, b


def evaluate_policies(g, alpha, beta, W=None, solver: str = "direct",
                      v_start: Optional[np.ndarray] = None) -> np.ndarray:
    """Value of the pair (alpha, beta) (Sec. 4.2, eq. (LSPI)).

    solver="direct": sparse LU + one refinement step.
    solver="krylov": for systems whose LU fill does not fit in memory (3-D
    grids of millions of states).  BiCGSTAB from `v_start` to a relative
    residual of 1e-14, then FP64 residual re-checks with correction solves
    until ||b - Av||_inf <= 1e-14 max(||b||_inf, ||v||_inf).  A reading, not
    the paper's sparse direct solve; the fixed point it serves is the same.
    """
    A, b = policy_system(g, alpha, beta, W)
    if solver == "direct":
        lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A")
        v = lu.solve(b)
        v += lu.solve(b - A @ v)
        return v
    if solver != "krylov":
        raise ValueError(f"unknown solver {solver!r}")
    v = np.zeros(g.n) if v_start is None else np.asarray(v_start, dtype=np.float64).copy()
    for _ in range(8):
        r = b - A @ v
        tol = 1e-14 * max(np.abs(b).max(initial=0.0), np.abs(v).max(initial=0.0))
        if np.abs(r).max(initial=0.0) <= tol:
            return v
        # a breakdown (info < 0) still returns its last iterate; the FP64
        # re-check above decides whether the correction was good enough
        e, _ = spla.bicgstab(A, r, rtol=1e-14, atol=0.0, maxiter=20000)
        v += e
    raise RuntimeError("Krylov policy evaluation did not reach the FP64 residual bound")


def _improve(g, Q, scale, alpha, beta):
    """One improvement sweep with the keep-the-incumbent tie rule.

    Returns (beta_in, F, alpha_out, beta_out):
      beta_in  -- MIN's improved policy at the current alpha (algo-MDP step 2),
      F        -- F(v) (eq. (eq1)),
      alpha_out, beta_out -- MAX's improved policy (PIalgo step 2) and MIN's
                  argmin at it.
    """
    n = g.n
    xs = np.arange(n)
    valid = _valid(g)
    Qb = np.where(valid, Q, np.inf)                     # for minima over b
    sb = np.where(valid, scale, 0.0)

    def argmin_keep(a_pol, b_inc):
        Qa = Qb[xs, a_pol, :]                           # (n, m2)
        mn = Qa.min(axis=1)
        tau = TIE_ULPS * EPS64 * sb[xs, a_pol, :].max(axis=1)
        low = np.argmin(Qa, axis=1)
        keep = (b_inc >= 0) & (Qa[xs, np.maximum(b_inc, 0)] <= mn + tau)
        return np.where(keep, b_inc, low).astype(np.int32), mn

    beta_in, _ = argmin_keep(alpha, beta)

    inner = Qb.min(axis=2)                              # (n, m1), +inf if a invalid
    inner = np.where(np.isinf(inner), -np.inf, inner)
    F = inner.max(axis=1)
    tau_out = TIE_ULPS * EPS64 * sb.max(axis=(1, 2))
    low_a = np.argmax(inner, axis=1)
    keep_a = inner[xs, alpha] >= F - tau_out
    alpha_out = np.where(keep_a, alpha, low_a).astype(np.int32)
    # MIN's answer at the new alpha: keep the incumbent where alpha is unchanged
    b_inc = np.where(alpha_out == alpha, beta, -1)
    beta_out, _ = argmin_keep(alpha_out, b_inc)
    return beta_in, F, alpha_out, beta_out


def policy_iteration(g, alpha0=None, beta0=None, v0=None, eps: float = 0.0,
                     max_outer: int = 10000, max_inner: int = 10000,
                     exact: Optional[np.ndarray] = None,
                     solver: str = "direct") -> OracleResult:
    """Hoffman-Karp / Puri policy iteration (Sec. 4.2, Algorithm PIalgo).

    The inner loop is Howard's algorithm for MIN at fixed alpha (Sec. 4.1,
    Algorithm algo-MDP).  After every value step the residual
    ||F(v) - v||_inf is computed and the iteration stops when it is <= eps
    (Sec. 5.1); with eps = 0 it stops when neither policy improves.
    """
    t0 = time.perf_counter()
    W = transition_matrix(g)
    n = g.n
    v = np.zeros(n) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    ga, gb = greedy(g, v, W)
    alpha = ga if alpha0 is None else np.asarray(alpha0, dtype=np.int32).copy()
    if beta0 is None:
        # MIN's greedy answer to alpha at v0 (lowest index on ties)
        Q, _ = q_values(g, v, W)
        Qa = np.where(_valid(g), Q, np.inf)[np.arange(n), alpha, :]
        beta = np.argmin(Qa, axis=1).astype(np.int32)
    else:
        beta = np.asarray(beta0, dtype=np.int32).copy()
    log = []
    k = 0
    inner_total = 0
    converged = False
    res = np.inf
    prev_outer_v = None
    while k < max_outer:
        k += 1
        nk = 0
        prev_inner_v = None
        stop = False
        while True:
            nk += 1
            inner_total += 1
            v = evaluate_policies(g, alpha, beta, W, solver=solver, v_start=v)
            Q, scale = q_values(g, v, W)
            beta_in, F, alpha_out, beta_out = _improve(g, Q, scale, alpha, beta)
            res = float(np.max(np.abs(F - v))) if n else 0.0
            entry = dict(k=k, nk=nk, res_inf=res,
                         res_l2=float(np.sqrt(np.mean((F - v) ** 2))) if n else 0.0,
                         inner_monotone=(prev_inner_v is None
                                         or bool(np.all(v <= prev_inner_v + 1e-9 * (1 + np.abs(v))))))
            if exact is not None:
                entry["err_inf"] = float(np.max(np.abs(v - exact)))
                entry["err_l2"] = float(np.sqrt(np.mean((v - exact) ** 2)))
            log.append(entry)
            prev_inner_v = v
            if res <= eps:
                stop = True
                break
            if np.array_equal(beta_in, beta) or nk >= max_inner:
                break
            beta = beta_in
        log[-1]["outer_monotone"] = (prev_outer_v is None or
                                     bool(np.all(v >= prev_outer_v - 1e-9 * (1 + np.abs(v)))))
        prev_outer_v = v
        if stop:
            alpha, beta = alpha_out, beta_out
            converged = True
            break
        if np.array_equal(alpha_out, alpha):
            converged = True
            break
        alpha, beta = alpha_out, beta_out
    return OracleResult(v, alpha, beta, res, k, inner_total, log, converged,
                        time.perf_counter() - t0)


# ----------------------------------------------------------------------------
# FAMGpi transfers and the coarse-to-fine loop (Sec. 5.2, Algorithm algo-FAMGPI)
# ----------------------------------------------------------------------------

def _axis_weights(s_c: int, s_f: int):
    """For fine interior index i (1..s_f): left coarse node k (0..s_c) and weight t."""
    i = np.arange(1, s_f + 1, dtype=np.int64)
    num = i * (s_c + 1)
    den = s_f + 1
    k = num // den
    t = (num - k * den) / den
    return k, t


def interp_value(v_c: np.ndarray, grid_c, grid_f) -> np.ndarray:
    """Value interpolation I from the coarse to the fine grid (Sec. 5.2).

    Multilinear on the coarse grid extended by its Dirichlet nodes.
    """
    d, sc, sf = grid_c.dim, grid_c.s, grid_f.s
    ext = np.zeros((sc + 2,) * d)
    if grid_c.bvals is not None:
        ext = grid_c.bvals.reshape((sc + 2,) * d).copy()
    # interior values; arrays are indexed [x_d, ..., x_1] (x1 fastest in memory)
    ext[(slice(1, sc + 1),) * d] = v_c.reshape((sc,) * d)
    k, t = _axis_weights(sc, sf)
    out = ext
    for ax in range(d):
        # interpolate along array axis `ax`
        lo = np.take(out, k, axis=ax)
        hi = np.take(out, np.minimum(k + 1, sc + 1), axis=ax)
        shape = [1] * out.ndim
        shape[ax] = sf
        tt = t.reshape(shape)
        out = (1.0 - tt) * lo + tt * hi
    return out.reshape(-1)


def interp_policy(p_c: np.ndarray, grid_c, grid_f) -> np.ndarray:
    """Strategy interpolation U (Sec. 5.2): copy a nearby coarse node's action."""
    d, sc, sf = grid_c.dim, grid_c.s, grid_f.s
    k, _ = _axis_weights(sc, sf)
    kk = np.clip(k, 1, sc) - 1
    pc = p_c.reshape((sc,) * d)
    out = pc
    for ax in range(d):
        out = np.take(out, kk, axis=ax)
    return out.reshape(-1).astype(np.int32)


def famg_pi(levels: List, eps: float, c: float, alpha0=None, beta0=None,
            v0=None) -> List[OracleResult]:
    """FAMGpi: PI on each level coarse -> fine with eps_l = c h_l^2, transfers
    of (v, alpha, beta) by I and U, final level with eps (Sec. 5.2)."""
    results = []
    a, b, v = alpha0, beta0, v0
    for li, g in enumerate(levels):
        last = li == len(levels) - 1
        e = eps if last else c * g.grid.h ** 2
        res = policy_iteration(g, a, b, v, eps=e)
        results.append(res)
        if not last:
            gf = levels[li + 1]
            v = interp_value(res.v, g.grid, gf.grid)
            a = interp_policy(res.alpha, g.grid, gf.grid)
            b = interp_policy(res.beta, g.grid, gf.grid)
    return results


def tied_states(g, v: np.ndarray, alpha: np.ndarray, gap: float = 1e-10) -> np.ndarray:
    """States whose top two action values differ by less than `gap`.

    Over a for MAX's choice, or over b at alpha(x) for MIN's choice.
    """
    Q, _ = q_values(g, v)
    valid = _valid(g)
    Qb = np.where(valid, Q, np.inf)
    inner = Qb.min(axis=2)
    inner = np.where(np.isinf(inner), -np.inf, inner)
    tied = np.zeros(g.n, dtype=bool)
    if g.m1 > 1:
        srt = np.sort(inner, axis=1)
        tied |= (srt[:, -1] - srt[:, -2]) < gap
    if g.m2 > 1:
        Qa = Qb[np.arange(g.n), alpha, :]
        srt = np.sort(Qa, axis=1)
        tied |= (srt[:, 1] - srt[:, 0]) < gap
    return tied
