"""The compact matrix forms of the cycle -- the stencil form of the finest
level and 16-bit column offsets on the other levels -- are a storage choice
only (the relaxation sweeps, residuals and FP64 residual of the multigrid
cycle, Algorithm MGcycle, Sec. 4.3): each row's entries are summed in the
same order as from CSR with 32-bit columns, so solves are the same bit for
bit with them and without them.  The games cover 2-D and 3-D grids, an FAMGpi hierarchy, a
batch of games of different sizes (per-game offsets), both precisions, the
fused first sweeps (nu1 >= 2) and single first sweeps (nu1 = 1), W-cycles
and l1-Jacobi; a point cloud (no stencil) keeps CSR on its finest level.  The games
have more rows than the per-game tail kernel takes from the finest level
(it keeps the CSR form)."""
import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs, games
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)
STATS = ("outer", "inner_total", "cycles_total", "value_steps", "setups_full", "setups_refresh")


def solve_both(make_handles, solve):
    """Solves with the stencil form and with CSR only; returns both results
    and the smoothing bytes of each (the stencil form moves fewer)."""
    out = []
    try:
        for mode in (-1, 0):
            P.shapley_tune_stencil(mode)
            hs = make_handles()
            try:
                P.shapley_probe_enable("smooth", True)
                st = solve(hs)
                pr = P.shapley_probe_read("smooth")
                P.shapley_probe_enable("smooth", False)
                res = [(P.shapley_get_value(h), *P.shapley_get_policy(h)) for h in hs]
            finally:
                for h in hs:
                    P.shapley_game_destroy(h)
            out.append((st if isinstance(st, list) else [st], res, pr["bytes"]))
    finally:
        P.shapley_tune_stencil(-1)
    return out


def check_same(name, out):
    (st1, r1, b1), (st0, r0, b0) = out
    for (v1, a1, bb1), (v0, a0, bb0) in zip(r1, r0):
        assert np.array_equal(v1, v0) and np.array_equal(a1, a0) and np.array_equal(bb1, bb0), name
    for s1, s0 in zip(st1, st0):
        assert s1["converged"] == 1 and s0["converged"] == 1
        for k in STATS:
            assert s1[k] == s0[k], (name, k, s1[k], s0[k])
    log(f"  {name}: same solve bit for bit; smoothing bytes {b1:.3e} (stencil) vs {b0:.3e} (CSR)")
    assert b1 < b0, "the compact forms were not used"


SINGLE = [
    ("isaacs2d 65 mixed V(2,2)", lambda: configs.c3_game(5, 65, 0.4), dict(precision=P.SHAPLEY_MIXED)),
    ("isaacs2d 65 fp64 V(2,2)", lambda: configs.c0(s=65), dict(precision=P.SHAPLEY_FP64)),
    ("isaacs2d 129 mixed V(1,1)", lambda: configs.c3_game(9, 129, 2.0),
     dict(precision=P.SHAPLEY_MIXED, nu1=1, nu2=1)),
    ("isaacs2d 129 mixed W(1,1) l1", lambda: configs.c3_game(2, 129, 0.2),
     dict(precision=P.SHAPLEY_MIXED, nu1=1, nu2=1, gamma=2, smoother=P.SHAPLEY_SMOOTH_L1)),
    ("isaacs3d 17 mixed", lambda: configs.c2(s=17), dict(precision=P.SHAPLEY_MIXED)),
    ("isaacs3d 33 fp64", lambda: configs.c2(s=33), dict(precision=P.SHAPLEY_FP64)),
]


@pytest.mark.parametrize("name,make,opts", SINGLE, ids=[c[0] for c in SINGLE])
def test_stencil_form_single_game(name, make, opts):
    g = make()
    out = solve_both(lambda: [P.create_from(g)],
                     lambda hs: P.shapley_solve(hs[0], P.shapley_default_opts(eps=1e-10, **opts, **LIMITS)))
    check_same(name, out)


def test_stencil_form_batch_of_sizes():
    gs = [configs.c3_game(k, side, lam) for k, (side, lam) in
          enumerate([(65, 0.3), (129, 3.0), (97, 1.0), (65, 8.0), (257, 0.15), (33, 0.5)])]
    out = solve_both(lambda: [P.create_from(g) for g in gs],
                     lambda hs: P.shapley_solve_batch(hs, P.shapley_default_opts(
                         eps=1e-9, precision=P.SHAPLEY_MIXED, forcing=0.2, **LIMITS)))
    check_same("batch of 6 games, sides 33..257", out)


def test_stencil_form_famg_hierarchy():
    lv = configs.c1_levels(points=257, coarsest_points=33)
    a0 = np.zeros(lv[0].n, np.int32)

    def make():
        return [P.shapley_game_create_hierarchy([P.create_from(x) for x in lv])]

    out = solve_both(make, lambda hs: P.shapley_solve(hs[0], P.shapley_default_opts(
        eps=1e-9, precision=P.SHAPLEY_MIXED, method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0, **LIMITS)))
    check_same("obstacle 257 FAMGpi", out)


def test_point_cloud_keeps_csr():
    g = games.point_cloud_game(1 << 13, 5)
    out = solve_both(lambda: [P.create_from(g)],
                     lambda hs: P.shapley_solve(hs[0], P.shapley_default_opts(
                         eps=1e-9, precision=P.SHAPLEY_MIXED, **LIMITS)))
    check_same("point cloud 2^13", out)
