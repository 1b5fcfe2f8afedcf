"""The refinement cycle replayed from a captured HIP graph gives exactly the
launch-by-launch results: every replay of several solves (each with its own
eager work and synchronisations between replays) is compared bit for bit
with the eager solve, for single games, a batch and FAMGpi grids."""
import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)


def run_single(g, graph, reps, **kw):
    h = P.create_from(g)
    try:
        out = []
        for _ in range(reps):
            st = P.shapley_solve(h, P.shapley_default_opts(graph=graph, **kw, **LIMITS))
            out.append((P.shapley_get_value(h), *P.shapley_get_policy(h), st["cycles_total"], st["outer"]))
        return out
    finally:
        P.shapley_game_destroy(h)


def same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    assert a[3:] == b[3:]


@pytest.mark.parametrize("variant", [dict(precision=P.SHAPLEY_FP64), dict(precision=P.SHAPLEY_MIXED),
                                     dict(precision=P.SHAPLEY_MIXED, eps=1e-8, forcing=0.1),
                                     dict(smoother=P.SHAPLEY_SMOOTH_CF, gamma=2, nu1=1, nu2=1)],
                         ids=["fp64", "mixed", "mixed-inexact", "cf-W"])
def test_graph_replays_equal_eager_single(variant):
    for g in (configs.c3_game(3, 129, 0.7), configs.c2(s=33)):
        eager = run_single(g, 0, 1, **variant)[0]
        for k, r in enumerate(run_single(g, 1, 3, **variant)):
            same(r, eager)
        log(f"  n={g.n} {variant}: 3 graph solves equal the eager one (cycles {eager[3]})")


def test_graph_replays_equal_eager_batch_and_famg():
    gs = [configs.c3_game(k, s, lam) for k, (s, lam) in enumerate([(65, 0.2), (129, 3.0), (97, 1.0), (65, 8.0)])]
    hs = [P.create_from(g) for g in gs]
    try:
        res = {}
        for graph in (0, 1, 1):
            st = P.shapley_solve_batch(hs, P.shapley_default_opts(precision=P.SHAPLEY_MIXED, graph=graph, **LIMITS))
            res.setdefault(graph, []).append(([P.shapley_get_value(h) for h in hs], [s["cycles_total"] for s in st]))
        for vals, cyc in res[1]:
            assert cyc == res[0][0][1]
            for a, b in zip(vals, res[0][0][0]):
                np.testing.assert_array_equal(a, b)
    finally:
        for h in hs:
            P.shapley_game_destroy(h)
    levels = configs.c1_levels(points=257, coarsest_points=33)
    H = P.shapley_game_create_hierarchy([P.create_from(x) for x in levels])
    try:
        a0 = np.zeros(levels[0].n, np.int32)
        out = []
        for graph in (0, 1, 1):
            st = P.shapley_solve(H, P.shapley_default_opts(method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0, graph=graph,
                                                           **LIMITS))
            out.append((P.shapley_get_value(H), *P.shapley_get_policy(H), st["cycles_total"], st["outer"]))
        same(out[1], out[0])
        same(out[2], out[0])
        log(f"  batch and FAMGpi: graph replays equal the eager solves (FAMG cycles {out[0][3]})")
    finally:
        P.shapley_game_destroy(H)
