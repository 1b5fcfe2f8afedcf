"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each check is computed by code that shares nothing with the oracle's
arithmetic: pure-Python value iteration, exhaustive policy enumeration with a
dense library solve, a linear program, closed forms, and the values the paper
prints for its 1-D worked example.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle
from shapley_inputs import configs, games
from shapley_inputs.games import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent helpers (pure Python / library routines)
# ---------------------------------------------------------------------------

def rows_of(g):
    """Python list of (cols, weights) per row -- plain loops, no SciPy."""
    out = []
    for i in range(g.nrows):
        a, b = int(g.row_ptr[i]), int(g.row_ptr[i + 1])
        out.append((g.col[a:b].tolist(), g.w[a:b].tolist()))
    return out


def valid_of(g, x, a, b):
    if g.valid is None:
        return True
    return bool(g.valid[(x * g.m1 + a) * g.m2 + b])


def bellman_loop(g, rows, v):
    """max over a of min over b of (r + mu * sum w v), written as loops (eq1)."""
    out = []
    for x in range(g.n):
        best = -math.inf
        for a in range(g.m1):
            worst = math.inf
            for b in range(g.m2):
                if not valid_of(g, x, a, b):
                    continue
                i = (x * g.m1 + a) * g.m2 + b
                cols, ws = rows[i]
                val = g.r[i] + g.mu * sum(w * v[c] for c, w in zip(cols, ws))
                worst = min(worst, val)
            if worst < math.inf:
                best = max(best, worst)
        out.append(best)
    return out


def value_iteration(g, tol=1e-15, max_it=100000):
    rows = rows_of(g)
    v = [0.0] * g.n
    for _ in range(max_it):
        nv = bellman_loop(g, rows, v)
        d = max(abs(p - q) for p, q in zip(nv, v))
        v = nv
        if d <= tol:
            break
    return np.array(v)


def dense_policy_value(g, alpha, beta):
    """Value of fixed policies via numpy.linalg.solve on the dense system."""
    M = np.zeros((g.n, g.n))
    rr = np.zeros(g.n)
    for x in range(g.n):
        i = (x * g.m1 + alpha[x]) * g.m2 + beta[x]
        for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
            M[x, g.col[k]] += g.w[k]
        rr[x] = g.r[i]
    return np.linalg.solve(np.eye(g.n) - g.mu * M, rr)


# ---------------------------------------------------------------------------
# the paper's worked example (Sec. 6.3)
# ---------------------------------------------------------------------------

def test_two_stopper_matches_paper_printed_errors():
    """1-D two-stopper game on 2049 points: the paper prints ||e||_inf = 1.16e-7,
    ||e||_L2 = 7.40e-8 and ||r_v||_inf = 1.11e-16 at convergence (Sec. 6.3)."""
    fx = json.load(open(os.path.join(GOLDEN, "two_stopper_2049.json")))
    pts = fx["points"]
    g = games.two_stopper_game(pts)
    m = pts - 1
    x = np.arange(1, m) / m
    u = games.two_stopper_exact(x)
    res = oracle.policy_iteration(g, exact=u)
    assert res.converged
    last = res.log[-1]
    pr = fx["printed"]
    assert float(f"{last['err_inf']:.2e}") == pytest.approx(pr["err_inf"], rel=1e-12)
    assert float(f"{last['err_l2']:.2e}") == pytest.approx(pr["err_l2"], rel=1e-12)
    assert last["res_inf"] <= 2 * pr["res_inf_upper"]
    # optimal strategies: MAX stops iff x > 0.91, MIN stops iff x < 0.09 (+-1 cell)
    th = fx["policy_thresholds"]
    h = 1.0 / m
    stop_max = res.alpha == 0
    assert np.all(stop_max[x > th["max_stops_above"] + h])
    assert not np.any(stop_max[x < th["max_stops_above"] - h])
    cont = ~stop_max
    stop_min = (res.beta == 0) & cont
    assert np.all(stop_min[(x < th["min_stops_below"] - h)])
    assert not np.any(stop_min[(x > th["min_stops_below"] + h) & cont])
    assert games.two_stopper_psi_bar() == pytest.approx(fx["psi_bar_approx"], abs=5e-3)


def test_two_stopper_psi_bar_closed_form():
    """psi_bar makes the closed form continuous at 0.91 (smooth fit, Sec. 6.3)."""
    pb = games.two_stopper_psi_bar()
    u = games.two_stopper_exact(np.array([0.09, 0.91 - 1e-12, 0.91 + 1e-12]))
    assert u[0] == pytest.approx(pb, abs=1e-12)
    assert u[1] == pytest.approx(-pb, abs=1e-9)


# ---------------------------------------------------------------------------
# brute force on tiny games
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,m1,m2,inv", [(0, 4, 2, 3, 0.0), (1, 6, 3, 2, 0.0),
                                               (2, 5, 3, 3, 0.3), (3, 3, 1, 4, 0.0),
                                               (4, 7, 4, 1, 0.0), (5, 5, 2, 2, 0.25)])
def test_oracle_matches_value_iteration(seed, n, m1, m2, inv):
    g = games.random_game(n, m1, m2, seed, mu=0.85, invalid_frac=inv)
    res = oracle.policy_iteration(g)
    v_vi = value_iteration(g)
    assert res.converged
    np.testing.assert_allclose(res.v, v_vi, rtol=0, atol=1e-12 * (1 + np.abs(v_vi).max()))
    # fixed point of the operator written as loops
    F = np.array(bellman_loop(g, rows_of(g), res.v))
    assert np.max(np.abs(F - res.v)) <= 1e-13 * (1 + np.abs(res.v).max())


@pytest.mark.parametrize("seed,n,m1,m2", [(10, 3, 2, 2), (11, 3, 2, 3), (12, 4, 2, 2), (13, 3, 3, 2)])
def test_oracle_matches_exhaustive_enumeration(seed, n, m1, m2):
    """v* = max over alpha of min over beta of v^{alpha beta}, componentwise:
    pure stationary optimal strategies exist (Sec. 2, Theorem)."""
    g = games.random_game(n, m1, m2, seed, mu=0.9)
    best = np.full(n, -np.inf)
    for alpha in itertools.product(range(m1), repeat=n):
        worst = np.full(n, np.inf)
        for beta in itertools.product(range(m2), repeat=n):
            worst = np.minimum(worst, dense_policy_value(g, alpha, beta))
        best = np.maximum(best, worst)
    res = oracle.policy_iteration(g)
    np.testing.assert_allclose(res.v, best, rtol=0, atol=1e-12)
    # the returned policies attain v*
    np.testing.assert_allclose(dense_policy_value(g, res.alpha, res.beta), best, atol=1e-12)


@pytest.mark.parametrize("seed", [20, 21, 22])
def test_one_player_matches_linear_program(seed):
    """m1 = 1 is Howard's MDP (Sec. 4.1): its value is the largest v with
    v <= r_b + mu P_b v for every b, a linear program."""
    n, m2 = 6, 3
    g = games.random_game(n, 1, m2, seed, mu=0.8)
    A_ub, b_ub = [], []
    for x in range(n):
        for b in range(m2):
            i = x * m2 + b
            row = np.zeros(n)
            row[x] = 1.0
            for k in range(g.row_ptr[i], g.row_ptr[i + 1]):
                row[g.col[k]] -= g.mu * g.w[k]
            A_ub.append(row)
            b_ub.append(g.r[i])
    lp = linprog(-np.ones(n), A_ub=np.array(A_ub), b_ub=np.array(b_ub),
                 bounds=[(None, None)] * n, method="highs")
    assert lp.status == 0
    res = oracle.policy_iteration(g)
    np.testing.assert_allclose(res.v, lp.x, atol=1e-9)


# ---------------------------------------------------------------------------
# greedy selectors and the tie rule.  argmax and argmin are sets (Sec. 2); the
# reading used by both sides: the lowest index attaining the extremum, and in
# policy iteration (Algorithm algo-MDP step 2, Algorithm PIalgo step 2) the
# incumbent kept unless another action beats it by more than a rounding bound.
# Exact ties are planted by copying an action (its rows repeat bit for bit).
# ---------------------------------------------------------------------------

def q_loops(g, v):
    """Q[x][a][b] = r + mu sum w v by plain loops (None for invalid pairs)."""
    rows = rows_of(g)
    Q = []
    for x in range(g.n):
        Qa = []
        for a in range(g.m1):
            Qb = []
            for b in range(g.m2):
                if not valid_of(g, x, a, b):
                    Qb.append(None)
                    continue
                i = (x * g.m1 + a) * g.m2 + b
                cols, ws = rows[i]
                Qb.append(g.r[i] + g.mu * sum(w * v[c] for c, w in zip(cols, ws)))
            Qa.append(Qb)
        Q.append(Qa)
    return Q


def lowest_argmin(vals):
    best, arg = math.inf, -1
    for k, q in enumerate(vals):
        if q is not None and q < best:
            best, arg = q, k
    return arg, best


def greedy_loops(g, v):
    """Lowest-index argmax_a min_b Q and the lowest-index argmin_b at it."""
    Q = q_loops(g, v)
    alpha, beta = [], []
    for x in range(g.n):
        best, ba = -math.inf, -1
        for a in range(g.m1):
            _, mn = lowest_argmin(Q[x][a])
            if mn < math.inf and mn > best:
                best, ba = mn, a
        alpha.append(ba)
        beta.append(lowest_argmin(Q[x][ba])[0])
    return np.array(alpha), np.array(beta)


def tie_game(seed, n=40, inv=0.0):
    """MAX's action 2 repeats its action 0; MIN's new action 1 repeats its old
    action 2, which moves to index 3 (the copy has the lower index)."""
    base = games.random_game(n, 2, 3, seed, mu=0.9, density=0.3, invalid_frac=inv)
    return games.with_copied_action(games.with_copied_action(base, 1, 0, 2), 2, 2, 1)


@pytest.mark.parametrize("seed,inv", [(50, 0.0), (51, 0.25), (52, 0.4)])
def test_greedy_matches_plain_loops_with_invalid_actions_and_ties(seed, inv):
    g = tie_game(seed, inv=inv)
    rng = np.random.default_rng(seed)
    ties_a = ties_b = 0
    for _ in range(4):
        v = rng.normal(size=g.n)
        a_ref, b_ref = greedy_loops(g, v)
        a, b = oracle.greedy(g, v)
        np.testing.assert_array_equal(a, a_ref)
        np.testing.assert_array_equal(b, b_ref)
        Q = q_loops(g, v)
        for x in range(g.n):
            inner = [lowest_argmin(Q[x][k])[1] for k in range(g.m1)]
            ties_a += inner[0] == max(inner) and inner[0] < math.inf
            qa = Q[x][a_ref[x]]
            ties_b += qa[1] is not None and qa[1] == lowest_argmin(qa)[1]
            assert qa[1] == qa[3]
        # chosen actions are valid and attain the extremum
        for x in range(g.n):
            assert valid_of(g, x, a[x], b[x])
    assert ties_a > 0 and ties_b > 0   # the planted ties were exercised


def test_improve_keeps_incumbent_at_planted_ties():
    """With (alpha, beta) incumbents: a tied incumbent is kept, a strictly
    beaten one is replaced by the lowest index attaining the extremum, and MIN's
    answer at a changed alpha has no incumbent (lowest index)."""
    g = tie_game(60, n=60)
    rng = np.random.default_rng(60)
    v = rng.normal(size=g.n)
    Q = q_loops(g, v)
    Qo, scale = oracle.q_values(g, v)
    margin = 1e-9
    a_inc = np.zeros(g.n, np.int32)
    b_inc = np.zeros(g.n, np.int32)
    expect_a, expect_bin = {}, {}
    for x in range(g.n):
        inner = [lowest_argmin(Q[x][k])[1] for k in range(g.m1)]
        top = max(inner)
        if inner[0] == top and inner[1] < top - margin:
            a_inc[x] = 2 if x % 2 else 1           # tied copy kept / beaten action replaced by 0
            expect_a[x] = 2 if x % 2 else 0
        elif inner[1] == top and inner[0] < top - margin:
            a_inc[x] = 2
            expect_a[x] = 1
        else:
            a_inc[x] = 1
        qa = Q[x][a_inc[x]]
        mn = lowest_argmin(qa)[1]
        if qa[3] == mn and qa[0] > mn + margin:
            b_inc[x] = 3 if x % 2 else 0           # tied original kept / beaten b replaced by the copy (1)
            expect_bin[x] = 3 if x % 2 else 1
        else:
            b_inc[x] = lowest_argmin(qa)[0]
    beta_in, F, alpha_out, beta_out = oracle.shapley_oracle._improve(g, Qo, scale, a_inc, b_inc)
    assert len(expect_a) >= 10 and len(expect_bin) >= 10
    for x, e in expect_a.items():
        assert alpha_out[x] == e, x
    for x, e in expect_bin.items():
        assert beta_in[x] == e, x
    for x in range(g.n):
        assert F[x] == max(lowest_argmin(Q[x][k])[1] for k in range(g.m1))
        if alpha_out[x] != a_inc[x]:
            assert beta_out[x] == lowest_argmin(Q[x][alpha_out[x]])[0]
        else:
            assert beta_out[x] == beta_in[x]


@pytest.mark.parametrize("player", [1, 2])
def test_tie_tolerance_is_a_rounding_bound(player):
    """An incumbent worse by a few units in the last place is kept; one worse
    by 1e-9 is replaced (the copy is the incumbent, the original the best)."""
    base = games.random_game(40, 2, 2, 70 + player, mu=0.9, density=0.3)
    rng = np.random.default_rng(player)
    v = rng.normal(size=base.n)
    for dr, kept in ((4e-16, True), (1e-9, False)):
        # MAX prefers larger values, MIN smaller ones: the copy is worse by |dr|
        g = games.with_copied_action(base, player, 0, 2, dr=-dr if player == 1 else dr)
        Q = q_loops(g, v)
        Qo, scale = oracle.q_values(g, v)
        inc_a = np.full(g.n, 2 if player == 1 else 0, np.int32)
        inc_b = np.full(g.n, 2 if player == 2 else 0, np.int32)
        for x in range(g.n):
            if player == 2:
                inc_a[x] = 0
        beta_in, F, alpha_out, _ = oracle.shapley_oracle._improve(g, Qo, scale, inc_a, inc_b)
        checked = 0
        for x in range(g.n):
            if player == 1:
                inner = [lowest_argmin(Q[x][k])[1] for k in range(g.m1)]
                if inner[0] != max(inner[:2]) or inner[0] - inner[1] < 1e-6:
                    continue
                checked += 1
                assert alpha_out[x] == (2 if kept else 0)
            else:
                qa = Q[x][0]
                if qa[0] - qa[1] > -1e-6:
                    continue
                checked += 1
                assert beta_in[x] == (2 if kept else 0)
        assert checked >= 5


def test_copied_actions_leave_the_value_unchanged():
    """Adding a copy of an action changes no value of the game (eq. (eq1) takes
    the same max and min); the policies found attain v*."""
    base = games.random_game(25, 2, 3, 80, mu=0.9, density=0.3, invalid_frac=0.2)
    g = games.with_copied_action(games.with_copied_action(base, 1, 1, 0), 2, 0, 3)
    r0 = oracle.policy_iteration(base)
    r1 = oracle.policy_iteration(g)
    assert r0.converged and r1.converged
    np.testing.assert_allclose(r1.v, r0.v, rtol=0, atol=1e-12)
    np.testing.assert_allclose(dense_policy_value(g, r1.alpha, r1.beta), r0.v, atol=1e-12)


# ---------------------------------------------------------------------------
# the Isaacs example with continuous action sets (Sec. 6.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("row", json.load(open(os.path.join(GOLDEN, "iex1_printed.json")))["rows"],
                         ids=lambda r: f"{r['points']} points")
def test_iex1_errors_match_paper_tables(row):
    """Eq. (Iex1) with the scheme (Iex1d): with action sets that contain the
    discrete optimum, the error against the exact solution sin x1 sin x2 is the
    one the paper prints at its last policy iteration (Tables Iex1t1-Iex1t2),
    to within 3 %.  The residual test mirrors the paper's stop."""
    g = games.iex1_local_game(row["points"])
    res = oracle.policy_iteration(g, eps=1e-10)
    x1, x2 = games.grid_coords(g.grid)
    e = res.v - games.iex1_exact(x1, x2)
    err_inf, err_l2 = np.abs(e).max(), np.sqrt(np.mean(e ** 2))
    assert res.converged
    assert err_inf == pytest.approx(row["err_inf"], rel=0.03)
    assert err_l2 == pytest.approx(row["err_l2"], rel=0.03)
    # the optimal actions lie inside the local sets (not on their edges)
    assert np.mean((res.alpha == 0) | (res.alpha == g.m1 - 1)) < 0.01


def test_iex1_finite_action_sets_converge():
    """Fixed finite subsets of the unit disk (directions on its circle) and of
    R^2 (a grid): refining them brings the value toward the exact solution."""
    errs = []
    for dirs, bpa in ((4, 2), (8, 4), (16, 8)):
        g = games.iex1_game(33, a_dirs=dirs, b_per_axis=bpa)
        res = oracle.policy_iteration(g)
        x1, x2 = games.grid_coords(g.grid)
        errs.append(np.abs(res.v - games.iex1_exact(x1, x2)).max())
    assert errs[0] > errs[1] > errs[2]


# ---------------------------------------------------------------------------
# games without a grid
# ---------------------------------------------------------------------------

def test_point_cloud_game_is_a_substochastic_game():
    g = games.point_cloud_game(500, 4)
    sums = np.add.reduceat(g.w, g.row_ptr[:-1].astype(np.int64))
    assert np.all(g.w > 0) and np.all(sums < 1.0) and np.all(sums > 0.9)
    res = oracle.policy_iteration(g)
    assert res.converged
    # fixed point of the operator written as loops (Sec. 2, eq. (eq1))
    F = np.array(bellman_loop(g, rows_of(g), res.v))
    assert np.max(np.abs(F - res.v)) <= 1e-12 * (1 + np.abs(res.v).max())


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_torus_constant_reward_closed_form():
    """Periodic Isaacs game, r = r0 - 0.1a^2 + 0.1b^2: v = r0/lambda, unique
    optimal actions a = 0, b = 0 (gap 0.1 h^2 / D)."""
    s, lam, r0 = 24, 1.5, 0.7
    grid = Grid(2, s, periodic=True)
    g = games.isaacs_game(grid, np.full(grid.n, r0), lam)
    res = oracle.policy_iteration(g)
    np.testing.assert_allclose(res.v, r0 / lam, rtol=1e-12)
    assert np.all(res.alpha == 1) and np.all(res.beta == 1)
    assert not oracle.tied_states(g, res.v, res.alpha).any()


def test_dirichlet_1d_quadratic_closed_form():
    """0.5 v'' = -r0, v(0)=v(1)=0: v = r0 x (1-x), exact for the centred
    second difference (scheme (centre), Sec. 3.3)."""
    s, r0 = 63, 1.3
    g = games.dirichlet_1d_game(s, r0)
    res = oracle.policy_iteration(g)
    x = np.arange(1, s + 1) / (s + 1)
    np.testing.assert_allclose(res.v, r0 * x * (1 - x), rtol=1e-12, atol=1e-14)


def test_stochastic_constant_reward_closed_form():
    """Row-stochastic transitions, constant reward r0 and discount mu:
    v = r0 / (1 - mu) (Sec. 2, the discounted payoff of a constant stream)."""
    g = games.scale_rows_to_stochastic(games.random_game(8, 3, 3, 7, mu=0.75))
    g.r[:] = 2.5
    res = oracle.policy_iteration(g)
    np.testing.assert_allclose(res.v, 2.5 / 0.25, rtol=1e-12)


def test_manufactured_isaacs_first_order_convergence():
    """Upwind scheme (decent)-(centre) is monotone and consistent: with f built
    so that u = sin(pi x1) sin(pi x2) x1 solves the Isaacs PDE for finite
    actions, ||v_h - u||_inf decreases like O(h) (Sec. 3.3; manufactured
    solutions as in Sec. 6.1)."""
    lam = 1.0
    acts = np.array([-1.0, 0.0, 1.0])

    def u_and_derivs(x1, x2):
        s1, c1, s2, c2 = np.sin(np.pi * x1), np.cos(np.pi * x1), np.sin(np.pi * x2), np.cos(np.pi * x2)
        u = s1 * s2 * x1
        ux1 = (np.pi * c1 * x1 + s1) * s2
        ux2 = s1 * np.pi * c2 * x1
        lap = (-np.pi ** 2 * s1 * x1 + 2 * np.pi * c1) * s2 - np.pi ** 2 * s1 * s2 * x1
        return u, ux1, ux2, lap

    errs = []
    for s in (15, 31, 63):
        grid = Grid(2, s)
        x1, x2 = games.grid_coords(grid)
        u, ux1, ux2, lap = u_and_derivs(x1, x2)
        # max_a (a u_x1 - 0.1 a^2) + min_b (b u_x2 + 0.1 b^2)
        ha = np.max(acts[None, :] * ux1[:, None] - 0.1 * acts[None, :] ** 2, axis=1)
        hb = np.min(acts[None, :] * ux2[:, None] + 0.1 * acts[None, :] ** 2, axis=1)
        f = -(0.5 * lap - lam * u + ha + hb)
        g = games.isaacs_game(grid, f, lam)
        res = oracle.policy_iteration(g)
        errs.append(np.max(np.abs(res.v - u)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 1.6 and errs[0] / errs[1] > 1.6


# ---------------------------------------------------------------------------
# operator properties and invariants
# ---------------------------------------------------------------------------

def test_operator_monotone_and_contracting():
    """F is monotone and mu-contracting in the sup-norm (Sec. 2)."""
    rng = np.random.default_rng(5)
    for seed in range(5):
        g = games.random_game(9, 3, 3, 100 + seed, mu=0.7, invalid_frac=0.2)
        for _ in range(10):
            v = rng.normal(size=g.n)
            w = rng.normal(size=g.n)
            Fv = oracle.shapley_operator(g, v)
            Fw = oracle.shapley_operator(g, w)
            assert np.max(np.abs(Fv - Fw)) <= g.mu * np.max(np.abs(v - w)) * (1 + 1e-12)
            hi = np.maximum(v, w)
            assert np.all(oracle.shapley_operator(g, hi) >= np.maximum(Fv, Fw) - 1e-12)
        # loops agree with the vectorised operator
        v = rng.normal(size=g.n)
        np.testing.assert_allclose(oracle.shapley_operator(g, v), bellman_loop(g, rows_of(g), v),
                                   atol=1e-13)


def test_policy_iteration_value_monotonicity_c0_small():
    """Outer values are non-decreasing, inner values non-increasing (Sec. 4.2)."""
    g = configs.c0(s=17)
    res = oracle.policy_iteration(g)
    assert res.converged
    assert all(e["inner_monotone"] for e in res.log)
    assert all(e.get("outer_monotone", True) for e in res.log)


def test_one_action_game_is_one_linear_solve():
    """m1 = m2 = 1: PI reduces to one solve of (LSPI) (Sec. 4.2)."""
    g = games.random_game(12, 1, 1, 31, mu=0.95)
    res = oracle.policy_iteration(g)
    assert res.inner_total == 1 and res.outer == 1
    v = dense_policy_value(g, np.zeros(12, int), np.zeros(12, int))
    np.testing.assert_allclose(res.v, v, atol=1e-13)
    A, b = oracle.policy_system(g, res.alpha, res.beta)
    assert np.max(np.abs(A @ res.v - b)) <= 1e-13 * np.max(np.abs(b))


def test_obstacle_complementarity():
    """Discrete form of the variational inequality (Sec. 3.2, eq. (visympli)):
    v >= psi, v >= cont(v), and one of them holds with equality everywhere."""
    g = configs.c1(points=65)
    res = oracle.policy_iteration(g)
    Q, _ = oracle.q_values(g, res.v)
    psi, cont = Q[:, 0, 0], Q[:, 1, 0]
    scale = 1e-12 * (1 + np.abs(res.v).max())
    assert np.all(res.v >= psi - scale) and np.all(res.v >= cont - scale)
    assert np.max(np.abs(np.minimum(res.v - psi, res.v - cont))) <= scale
    frac = np.mean(res.alpha == 0)
    assert 0.2 <= frac <= 0.8, frac


def test_obstacle_starting_from_stop_everywhere():
    """C1 starts with MAX stopping everywhere (Sec. 6.2); same fixed point."""
    g = configs.c1(points=33)
    a = oracle.policy_iteration(g)
    b = oracle.policy_iteration(g, alpha0=np.zeros(g.n, np.int32), beta0=np.zeros(g.n, np.int32))
    np.testing.assert_allclose(a.v, b.v, atol=1e-13)


# ---------------------------------------------------------------------------
# FAMGpi transfers (Sec. 5.2)
# ---------------------------------------------------------------------------

def paper_interp(v_c, grid_c, grid_f):
    """I of Sec. 5.2 written out: fine nodes that are coarse nodes copy, the
    others average the coarse nodes (Dirichlet nodes included, at their
    boundary values) within Euclidean distance h_l."""
    d, sc, sf = grid_c.dim, grid_c.s, grid_f.s
    hc = 1.0 / (sc + 1)
    hf = 1.0 / (sf + 1)
    bv = grid_c.bvals if grid_c.bvals is not None else np.zeros((sc + 2) ** d)
    out = np.zeros(sf ** d)
    for xf in range(sf ** d):
        idx = [(xf // sf ** k) % sf + 1 for k in range(d)]
        pos = [i * hf for i in idx]
        acc, cnt = 0.0, 0
        for cidx in itertools.product(range(sc + 2), repeat=d):
            cpos = [c * hc for c in cidx]
            dist = math.sqrt(sum((p - q) ** 2 for p, q in zip(pos, cpos)))
            if dist <= hc * (1 + 1e-9):
                if dist < 1e-12:
                    acc, cnt = None, 0
                    inner = all(1 <= c <= sc for c in cidx)
                    lin = sum((c - 1) * sc ** k for k, c in enumerate(cidx))
                    out[xf] = v_c[lin] if inner else bv[sum(c * (sc + 2) ** k for k, c in enumerate(cidx))]
                    break
                inner = all(1 <= c <= sc for c in cidx)
                if inner:
                    acc += v_c[sum((c - 1) * sc ** k for k, c in enumerate(cidx))]
                else:
                    acc += bv[sum(c * (sc + 2) ** k for k, c in enumerate(cidx))]
                cnt += 1
        if acc is not None:
            out[xf] = acc / cnt
    return out


@pytest.mark.parametrize("dim,sc", [(1, 7), (2, 3), (2, 7), (3, 3)])
def test_interp_value_is_the_paper_neighbour_average(dim, sc):
    rng = np.random.default_rng(dim * 10 + sc)
    sf = 2 * (sc + 1) - 1
    bv = rng.normal(size=(sc + 2) ** dim)
    gc = Grid(dim, sc, bvals=bv)
    gf = Grid(dim, sf)
    v_c = rng.normal(size=sc ** dim)
    np.testing.assert_allclose(oracle.interp_value(v_c, gc, gf), paper_interp(v_c, gc, gf),
                               atol=1e-14)


def test_interp_policy_copies_coarse_nodes():
    gc, gf = Grid(2, 7), Grid(2, 15)
    p = np.arange(49, dtype=np.int32) % 3
    q = oracle.interp_policy(p, gc, gf).reshape(15, 15)
    pc = p.reshape(7, 7)
    # fine nodes that are coarse nodes copy exactly
    np.testing.assert_array_equal(q[1::2, 1::2], pc)


def test_famg_matches_single_level_fixed_point():
    """FAMGpi reaches the same unique fixed point as PI on the finest grid."""
    levels = configs.c1_levels(points=129, coarsest_points=17)
    res = oracle.famg_pi(levels, eps=0.0, c=1e-2)
    ref = oracle.policy_iteration(levels[-1])
    np.testing.assert_allclose(res[-1].v, ref.v, atol=1e-13)
    np.testing.assert_array_equal(res[-1].alpha, ref.alpha)


# ---------------------------------------------------------------------------
# the Krylov policy evaluation used where the sparse LU does not fit (3-D)
# ---------------------------------------------------------------------------

def test_krylov_evaluation_matches_dense_solve():
    """BiCGSTAB + FP64 re-checks equals numpy's dense solve of (LSPI)."""
    g = configs.c2(s=5)
    rng = np.random.default_rng(11)
    alpha = rng.integers(0, g.m1, g.n).astype(np.int32)
    beta = rng.integers(0, g.m2, g.n).astype(np.int32)
    v = oracle.evaluate_policies(g, alpha, beta, solver="krylov")
    ref = dense_policy_value(g, alpha, beta)
    np.testing.assert_allclose(v, ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())


def test_krylov_policy_iteration_matches_value_iteration_3d():
    """3-D Isaacs game (the workload family where the Krylov path is used):
    policy iteration with Krylov evaluations reaches the fixed point found by
    pure-Python value iteration."""
    grid = Grid(3, 4)
    rng = np.random.default_rng(5)
    f = rng.uniform(-1.0, 1.0, grid.n)
    g = games.isaacs_game(grid, f, 5.0)
    res = oracle.policy_iteration(g, solver="krylov")
    assert res.converged
    vi = value_iteration(g)
    np.testing.assert_allclose(res.v, vi, rtol=1e-12, atol=1e-14)


def test_krylov_torus_closed_form():
    s, lam, r0 = 16, 0.3, -0.4
    grid = Grid(2, s, periodic=True)
    g = games.isaacs_game(grid, np.full(grid.n, r0), lam)
    res = oracle.policy_iteration(g, solver="krylov")
    np.testing.assert_allclose(res.v, r0 / lam, rtol=1e-12)
    assert np.all(res.alpha == 1) and np.all(res.beta == 1)
