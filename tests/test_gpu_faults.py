"""Error paths under injected device allocation failures (library
robustness, no passage of the paper): whichever allocation of game creation,
AMG setup or solve fails, the call returns SHAPLEY_ENOMEM, the handles stay
usable, and the same call repeated without the fault gives the result of an
undisturbed run bit for bit.  Covers a single game (AMGpi, FP32 cycles with
FP64 refinement), an FAMGpi hierarchy and a batch."""
import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)


def run(make, solve):
    hs = make()
    try:
        st = solve(hs)
        return st, [(P.shapley_get_value(h), *P.shapley_get_policy(h)) for h in hs]
    finally:
        for h in hs:
            P.shapley_game_destroy(h)


def inject_everywhere(what, make, solve, max_k=3000):
    """Fail the k-th allocation, k = 1, 2, ..., until a run makes fewer than
    k allocations; after each failure the call is repeated without it."""
    _, ref = run(make, solve)
    failures = 0
    for k in range(1, max_k):
        P.shapley_debug_fail_alloc(k)
        try:
            try:
                hs = make()
            except P.ShapleyError as e:
                assert e.code == P.SHAPLEY_ENOMEM and "allocation" in str(e), e
                failures += 1
                continue
            try:
                failed = False
                try:
                    solve(hs)
                except P.ShapleyError as e:
                    assert e.code == P.SHAPLEY_ENOMEM and "allocation" in str(e), e
                    failed = True
                P.shapley_debug_fail_alloc(0)
                solve(hs)  # the same handles, no fault
                out = [(P.shapley_get_value(h), *P.shapley_get_policy(h)) for h in hs]
            finally:
                for h in hs:
                    P.shapley_game_destroy(h)
        finally:
            P.shapley_debug_fail_alloc(0)
        for (v, a, b), (vr, ar, br) in zip(out, ref):
            np.testing.assert_array_equal(v, vr)
            np.testing.assert_array_equal(a, ar)
            np.testing.assert_array_equal(b, br)
        if failed:
            failures += 1
        else:
            log(f"  {what}: {failures} injected failures, each recovered; {k - 1} allocations in all")
            assert failures == k - 1
            return
    raise AssertionError(f"{what}: more than {max_k} allocations")


def create_all(games):
    """Handles of the games; on a failure the ones already made are destroyed."""
    hs = []
    try:
        for g in games:
            hs.append(P.create_from(g))
    except P.ShapleyError:
        for h in hs:
            P.shapley_game_destroy(h)
        raise
    return hs


def test_single_game_survives_allocation_failures():
    g = configs.c3_game(2, 33, 1.0)
    o = P.shapley_default_opts(precision=P.SHAPLEY_MIXED, **LIMITS)
    inject_everywhere("isaacs 33^2 mixed", lambda: create_all([g]), lambda hs: P.shapley_solve(hs[0], o))


def test_famg_hierarchy_survives_allocation_failures():
    lv = configs.c1_levels(points=65, coarsest_points=33)
    a0 = np.zeros(lv[0].n, np.int32)
    o = P.shapley_default_opts(method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0, **LIMITS)
    def make():
        levels = create_all(lv)
        try:
            return [P.shapley_game_create_hierarchy(levels)]
        except P.ShapleyError:
            for h in levels:
                P.shapley_game_destroy(h)
            raise

    inject_everywhere("obstacle 65 FAMGpi", make, lambda hs: P.shapley_solve(hs[0], o))


def test_batch_survives_allocation_failures():
    gs = [configs.c3_game(k, 17 + 16 * (k % 2), 0.5 + k) for k in range(4)]
    o = P.shapley_default_opts(precision=P.SHAPLEY_MIXED, **LIMITS)
    inject_everywhere("batch of 4", lambda: create_all(gs), lambda hs: P.shapley_solve_batch(hs, o))
