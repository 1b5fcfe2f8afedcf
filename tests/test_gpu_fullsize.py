"""Parity at the benchmark workloads' full sizes, in the launch shapes the
benchmark times, compared at every state.

* Obstacle problem, 1025 x 1025 points, FAMGpi: the oracle's FAMGpi fixed
  point is computed in worker processes while the GPU solves run.
* 3-D Isaacs game, 129^3 interior points: the oracle's fixed point at every
  state is stored (tests/golden/isaacs3d_129_full.npz, written by
  tests/golden/make_fullsize.py from the oracle alone; its Krylov policy
  evaluations take minutes).
* 256 2-D Isaacs games batched: all 256 against the oracle (worker processes).
* Serving: the first 16 requests of the serving stream through the server,
  all 16 against the oracle (worker processes).

Runs to the fixed point (eps = 0: no policy improves, exact linear solves)
are held to the parity bar (FP64 1e-9, mixed 1e-6 relative, policies equal
at untied states, extrema at tied ones).  Runs with the benchmark's stop
(||F(v) - v||_inf <= 1e-8) are held to what that stop guarantees: the
reported residual, and ||v - v*||_inf <= 1e-8 / (1 - mu_max), mu_max the
largest row sum of the game's substochastic weights (F is a
mu_max-contraction in the sup norm, Sec. 2).
"""
import json
import os
import types

import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import compare_with_oracle, log
from oracle.jobs import Jobs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BENCH = dict(max_outer=5000, max_inner=5000, forcing=0.2, reuse_frac=0.5)


def ref_of(d):
    return types.SimpleNamespace(v=np.asarray(d["v"], np.float64), alpha=np.asarray(d["alpha"], np.int32),
                                 beta=np.asarray(d["beta"], np.int32))


def load_full(name):
    """Oracle fixed point at every state (value truncated to 36 mantissa bits)."""
    with np.load(os.path.join(GOLDEN, name)) as d:
        n = int(d["n"])
        planes = d["v_planes"]
        b = np.zeros((n, 8), np.uint8)
        for k in range(planes.shape[0]):
            b[:, 7 - k] = planes[k]
        v = b.view(np.float64).reshape(-1).copy()
        return types.SimpleNamespace(v=v, alpha=d["alpha"].astype(np.int32), beta=d["beta"].astype(np.int32),
                                     tied=np.unpackbits(d["tied"])[:n].astype(bool), n=n)


def check_all(g, v, a, b, ref, tol, what):
    err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, tol)
    log(f"  {what}: rel err {err:.2e} (tol {tol:g}) over {g.n} states, policy mismatches {len(ma)}/{len(mb)}, "
        f"tied {int(tied.sum())}")
    assert err <= tol
    assert len(ma) == 0 and len(mb) == 0
    return err


def mu_max(g):
    csum = np.concatenate([[0.0], np.cumsum(g.w)])
    rows = csum[g.row_ptr[1:]] - csum[g.row_ptr[:-1]]
    return g.mu * float(rows.max())


def test_obstacle_1025_famg_full_size():
    jobs = Jobs([("c1", "c1", [1025, 33], 0.0)])
    levels = configs.c1_levels(points=1025, coarsest_points=33)
    g = levels[-1]
    hs = [P.create_from(x) for x in levels]
    H = P.shapley_game_create_hierarchy(hs)
    a0 = np.zeros(levels[0].n, np.int32)
    res = {}
    try:
        for name, prec, eps in (("fp64 fixed point", P.SHAPLEY_FP64, 0.0),
                                ("mixed fixed point", P.SHAPLEY_MIXED, 0.0),
                                ("fp64 bench stop", P.SHAPLEY_FP64, 1e-8),
                                ("mixed bench stop", P.SHAPLEY_MIXED, 1e-8)):
            log(f"obstacle 1025 FAMGpi {name}")
            o = P.shapley_default_opts(eps=eps, precision=prec, method=P.SHAPLEY_FAMGPI, alpha0=a0,
                                       beta0=a0, **BENCH)
            st = P.shapley_solve(H, o)
            res[name] = (P.shapley_get_value(H), *P.shapley_get_policy(H), st)
            log(f"  outer {st['outer']} residual {st['residual']:.2e} grids {st['fmg_levels']}")
            assert st["converged"] == 1
    finally:
        P.shapley_game_destroy(H)
    ref = ref_of(jobs.wait(timeout=300, log=log)["c1"])
    for name, (v, a, b, st) in res.items():
        if "fixed point" in name:
            check_all(g, v, a, b, ref, 1e-9 if "fp64" in name else 1e-6, name)
        else:
            assert st["residual"] <= 1e-8
            bound = 1e-8 / (1.0 - mu_max(g))
            err = np.max(np.abs(v - ref.v))
            log(f"  {name}: |v - v*| {err:.2e} over all states <= contraction bound {bound:.2e}")
            assert err <= bound
    d = np.max(np.abs(res["mixed bench stop"][0] - res["fp64 bench stop"][0])) / np.max(np.abs(ref.v))
    log(f"  mixed vs fp64 at the bench stop: {d:.2e}")
    assert d <= 1e-6


def test_isaacs3d_129_full_size():
    ref = load_full("isaacs3d_129_full.npz")
    g = configs.c2(s=129)
    assert g.n == ref.n
    h = P.create_from(g)
    try:
        for name, prec, eps, tol in (("fp64 fixed point", P.SHAPLEY_FP64, 0.0, 1e-9),
                                     ("mixed fixed point", P.SHAPLEY_MIXED, 0.0, 1e-6),
                                     ("mixed bench stop", P.SHAPLEY_MIXED, 1e-8, None)):
            log(f"isaacs3d 129 AMGpi {name}")
            o = P.shapley_default_opts(eps=eps, precision=prec, **BENCH)
            st = P.shapley_solve(h, o)
            v = P.shapley_get_value(h)
            a, b = P.shapley_get_policy(h)
            log(f"  outer {st['outer']} inner {st['inner_total']} residual {st['residual']:.2e} "
                f"levels {st['levels']} op complexity {st['op_complexity']:.2f}")
            assert st["converged"] == 1
            if tol is not None:
                check_all(g, v, a, b, ref, tol, name)
            else:
                assert st["residual"] <= 1e-8
                bound = 1e-8 / (1.0 - mu_max(g))
                err = np.max(np.abs(v - ref.v))
                log(f"  |v - v*| {err:.2e} over all states <= contraction bound {bound:.2e}")
                assert err <= bound
    finally:
        P.shapley_game_destroy(h)


def _c3_cost(job):
    side = job[2][1]
    return float(side) ** 3


def test_batch_256_games_full_size():
    side, lam = configs.c3_sizes(count=256)
    jobs = Jobs([(f"g{k}", "c3", [k, int(side[k]), float(lam[k])], 0.0) for k in range(256)], cost=_c3_cost)
    gs = [configs.c3_game(k, side[k], lam[k]) for k in range(256)]
    hs = [P.create_from(g) for g in gs]
    try:
        log(f"batch of 256 games, sum n = {sum(g.n for g in gs)}")
        st = P.shapley_solve_batch(hs, P.shapley_default_opts(precision=P.SHAPLEY_MIXED, **BENCH))
        assert all(s["converged"] == 1 for s in st)
        vals = [(P.shapley_get_value(h), *P.shapley_get_policy(h)) for h in hs]
        st2 = P.shapley_solve_batch(hs, P.shapley_default_opts(eps=1e-8, precision=P.SHAPLEY_MIXED, **BENCH))
        worst = max(s["residual"] for s in st2)
        stop_vals = [P.shapley_get_value(h) for h in hs]
        log(f"  bench stop: worst residual {worst:.2e}")
        assert all(s["converged"] == 1 for s in st2) and worst <= 1e-8
    finally:
        for h in hs:
            P.shapley_game_destroy(h)
    refs = jobs.wait(timeout=600, log=log)
    worst_err, worst_stop = 0.0, 0.0
    for k, g in enumerate(gs):
        ref = ref_of(refs[f"g{k}"])
        v, a, b = vals[k]
        err, ma, mb, _ = compare_with_oracle(g, v, a, b, ref, 1e-6)
        assert err <= 1e-6 and len(ma) == 0 and len(mb) == 0, (k, err, len(ma), len(mb))
        worst_err = max(worst_err, err)
        e2 = np.max(np.abs(stop_vals[k] - ref.v))
        assert e2 <= 1e-8 / (1.0 - mu_max(g)), k
        worst_stop = max(worst_stop, e2 / np.max(np.abs(ref.v)))
    log(f"  all 256 games: worst rel err {worst_err:.2e} at the fixed point, {worst_stop:.2e} at the bench stop")


def test_serving_stream_full_size():
    reqs = configs.c4_requests(count=1000)[:16]
    specs = []
    for i, (kind, side, lam, seed) in enumerate(reqs):
        specs.append((f"r{i}", "c4_isaacs", [int(side), float(lam), int(seed)], 0.0) if kind == 0 else
                     (f"r{i}", "c4_obstacle", [int(side), int(seed), float(lam)], 0.0))
    jobs = Jobs(specs, cost=lambda j: (j[2][0] ** 2) * (9 if j[1] == "c4_isaacs" else 2))
    handles = []
    for kind, side, lam, seed in reqs:
        if kind == 0:
            g = configs.c4_game(kind, side, lam, seed)
            handles.append((P.create_from(g), [g]))
        else:
            lv = configs.obstacle_levels_for_side(side, seed, lam)
            handles.append((P.shapley_game_create_hierarchy([P.create_from(x) for x in lv]), lv))
    srv = P.shapley_server_create(200 * 10 ** 9)
    try:
        tickets = []
        for (h, lv), (kind, side, lam, seed) in zip(handles, reqs):
            if kind == 0:
                o = P.shapley_default_opts(precision=P.SHAPLEY_MIXED, **BENCH)
            else:
                a0 = np.zeros(lv[0].n, np.int32)
                o = P.shapley_default_opts(precision=P.SHAPLEY_MIXED, method=P.SHAPLEY_FAMGPI, alpha0=a0,
                                           beta0=a0, **BENCH)
            tickets.append(P.shapley_server_submit(srv, h, o))
        steps = 0
        max_cohorts = 0
        while P.shapley_server_step(srv) > 0:
            steps += 1
            max_cohorts = max(max_cohorts, P.shapley_server_info(srv)["cohorts"])
            assert steps < 100000
        log(f"serving 16 requests: {steps} server steps, up to {max_cohorts} cohorts at once")
        results = []
        for (h, lv), t in zip(handles, tickets):
            st = P.shapley_server_poll(srv, t)
            assert st is not None and st["converged"] == 1
            results.append((P.shapley_get_value(h), *P.shapley_get_policy(h)))
    finally:
        P.shapley_server_destroy(srv)
        for h, _ in handles:
            P.shapley_game_destroy(h)
    refs = jobs.wait(timeout=600, log=log)
    for i, ((h, lv), (kind, side, lam, seed)) in enumerate(zip(handles, reqs)):
        v, a, b = results[i]
        err, ma, mb, _ = compare_with_oracle(lv[-1], v, a, b, ref_of(refs[f"r{i}"]), 1e-6)
        log(f"  request seed {seed} kind {kind} side {side}: rel err {err:.2e}")
        assert err <= 1e-6 and len(ma) == 0 and len(mb) == 0
