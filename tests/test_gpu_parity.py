"""End-to-end parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: final policies identical except at states whose top two action values
differ by less than 1e-10 at the oracle's value; values within 1e-9
(relative, sup-norm) in FP64 mode and 1e-6 in mixed mode.
"""
import numpy as np
import pytest

import oracle
import paper_1107_1653_amd as P
from shapley_inputs import configs, games
from tests.gpu_helpers import compare_with_oracle, log, solve_gpu

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)


@pytest.mark.parametrize("s", [9, 17, 33])
@pytest.mark.parametrize("prec,tol", [(P.SHAPLEY_FP64, 1e-9), (P.SHAPLEY_MIXED, 1e-6)])
def test_isaacs2d_c0_family(s, prec, tol):
    g = configs.c0(s=s)
    log(f"isaacs2d s={s} prec={prec}")
    ref = oracle.policy_iteration(g)
    v, a, b, st = solve_gpu(g, precision=prec, **LIMITS)
    err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, tol)
    log(f"  err {err:.2e} outer {st['outer']} inner {st['inner_total']} cycles {st['cycles_total']} "
        f"levels {st['levels']} tied {tied.sum()} (oracle {ref.outer}/{ref.inner_total})")
    assert st["converged"] == 1
    assert err <= tol
    assert len(ma) == 0 and len(mb) == 0


@pytest.mark.parametrize("seed,n,m1,m2,inv", [(0, 40, 2, 3, 0.0), (1, 60, 3, 2, 0.2), (2, 25, 1, 4, 0.0)])
def test_random_games_dense_path(seed, n, m1, m2, inv):
    """General (non-grid) games; n <= coarse_max exercises the dense solve."""
    g = games.random_game(n, m1, m2, seed, mu=0.9, density=0.2, invalid_frac=inv)
    log(f"random seed={seed} n={n}")
    ref = oracle.policy_iteration(g)
    v, a, b, st = solve_gpu(g, **LIMITS)
    err, ma, mb, _ = compare_with_oracle(g, v, a, b, ref, 1e-9)
    log(f"  err {err:.2e} outer {st['outer']} inner {st['inner_total']}")
    assert err <= 1e-9 and len(ma) == 0 and len(mb) == 0


@pytest.mark.parametrize("pts", [33, 65, 129])
def test_obstacle_amgpi_from_stop_everywhere(pts):
    g = configs.c1(points=pts)
    log(f"obstacle pts={pts}")
    a0 = np.zeros(g.n, np.int32)
    ref = oracle.policy_iteration(g, alpha0=a0, beta0=a0)
    v, a, b, st = solve_gpu(g, alpha0=a0, beta0=a0, **LIMITS)
    err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, 1e-9)
    log(f"  err {err:.2e} outer {st['outer']} (oracle {ref.outer}) levels {st['levels']}")
    assert st["converged"] == 1 and err <= 1e-9 and len(ma) == 0


def test_isaacs3d_small():
    g = configs.c2(s=17)
    log("isaacs3d s=17")
    ref = oracle.policy_iteration(g)
    for prec, tol in ((P.SHAPLEY_FP64, 1e-9), (P.SHAPLEY_MIXED, 1e-6)):
        v, a, b, st = solve_gpu(g, precision=prec, **LIMITS)
        err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, tol)
        log(f"  prec {prec} err {err:.2e} levels {st['levels']} cycles {st['cycles_total']}")
        assert err <= tol and len(ma) == 0 and len(mb) == 0


def test_two_stopper_paper_example_on_gpu():
    """Sec. 6.3 worked example: ||e||_inf = 1.16e-7 at 2049 points."""
    g = games.two_stopper_game(2049)
    x = np.arange(1, 2048) / 2048
    u = games.two_stopper_exact(x)
    v, a, b, st = solve_gpu(g, max_outer=2000, max_inner=2000)
    e = np.max(np.abs(v - u))
    log(f"two-stopper err_inf {e:.3e} outer {st['outer']}")
    assert float(f"{e:.2e}") == pytest.approx(1.16e-7)


def test_batch_matches_alone_and_oracle():
    """Batched lock-step solve (one launch per level for all games) gives each
    game the result it gets alone; both match the oracle."""
    gs = [configs.c3_game(k, side, lam) for k, (side, lam) in
          enumerate([(17, 0.3), (33, 5.0), (9, 1.0), (25, 0.1), (33, 9.0), (17, 2.0)])]
    gs.append(configs.c1(points=33))
    hs = [P.create_from(g) for g in gs]
    try:
        st = P.shapley_solve_batch(hs, P.shapley_default_opts(**LIMITS))
        vb = [P.shapley_get_value(h) for h in hs]
        pb = [P.shapley_get_policy(h) for h in hs]
    finally:
        for h in hs:
            P.shapley_game_destroy(h)
    for k, g in enumerate(gs):
        ref = oracle.policy_iteration(g)
        v, a, b, _ = solve_gpu(g, **LIMITS)
        err_alone = np.max(np.abs(vb[k] - v)) / np.max(np.abs(v))
        err, ma, mb, _ = compare_with_oracle(g, vb[k], pb[k][0], pb[k][1], ref, 1e-9)
        log(f"  game {k} n={g.n} batch-vs-alone {err_alone:.2e} vs-oracle {err:.2e} outer {st[k]['outer']}")
        assert err <= 1e-9 and len(ma) == 0 and len(mb) == 0
        assert err_alone <= 1e-12
        np.testing.assert_array_equal(pb[k][0], a)


def test_famg_hierarchy_matches_finest_oracle():
    """FAMGpi (Algorithm algo-FAMGPI) reaches the unique fixed point of the
    finest game (Sec. 5.2)."""
    levels = configs.c1_levels(points=129, coarsest_points=17)
    ref = oracle.policy_iteration(levels[-1])
    hs = [P.create_from(g) for g in levels]
    H = P.shapley_game_create_hierarchy(hs)
    try:
        a0 = np.zeros(levels[0].n, np.int32)
        for prec, tol in ((P.SHAPLEY_FP64, 1e-9), (P.SHAPLEY_MIXED, 1e-6)):
            o = P.shapley_default_opts(method=P.SHAPLEY_FAMGPI, precision=prec, alpha0=a0, beta0=a0, **LIMITS)
            st = P.shapley_solve(H, o)
            v = P.shapley_get_value(H)
            a, b = P.shapley_get_policy(H)
            err, ma, mb, _ = compare_with_oracle(levels[-1], v, a, b, ref, tol)
            log(f"  famg prec {prec} err {err:.2e} outer {st['outer']} fmg_levels {st['fmg_levels']}")
            assert err <= tol and len(ma) == 0
    finally:
        P.shapley_game_destroy(H)


def test_apply_operator_matches_oracle():
    """F(v) and greedy policies of the HIP sweep equal the oracle's eq1 at random v."""
    g = games.random_game(50, 3, 3, 77, mu=0.9, density=0.2, invalid_frac=0.2)
    h = P.create_from(g)
    try:
        rng = np.random.default_rng(0)
        for _ in range(3):
            v = rng.normal(size=g.n)
            F, a, b = P.shapley_apply_operator(h, v)
            Fo = oracle.shapley_operator(g, v)
            ao, bo = oracle.greedy(g, v)
            np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-13)
            np.testing.assert_array_equal(a, ao)
            np.testing.assert_array_equal(b, bo)
    finally:
        P.shapley_game_destroy(h)


def test_server_continuous_batching_matches_alone():
    """Requests that arrive while others run are admitted as budget frees up;
    each result is the one the game gets alone (and the oracle's)."""
    specs = [(0, 17, 0.5, 2001), (1, 31, 2.0, 2002), (0, 33, 9.0, 2003), (1, 15, 0.3, 2004),
             (0, 9, 1.0, 2005), (1, 33, 5.0, 2006)]
    gs = [configs.c4_game(*sp) for sp in specs]
    lv = configs.c1_levels(points=65, coarsest_points=17)
    hs = [P.create_from(g) for g in gs]
    H = P.shapley_game_create_hierarchy([P.create_from(g) for g in lv])
    sizes = [P.shapley_game_bytes(h) for h in hs]
    # a budget that holds about two requests at a time
    srv = P.shapley_server_create(int(3 * max(sizes) * 4))
    try:
        o = P.shapley_default_opts(**LIMITS)
        a0 = np.zeros(lv[0].n, np.int32)
        of = P.shapley_default_opts(method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0, **LIMITS)
        tickets = [P.shapley_server_submit(srv, hs[k], o) for k in range(3)]
        steps = 0
        max_active = 0
        while steps < 3:
            max_active = max(max_active, P.shapley_server_step(srv))
            steps += 1
        running_early = [t for t in tickets if P.shapley_server_poll(srv, t) is None]
        tickets += [P.shapley_server_submit(srv, hs[k], o) for k in range(3, 6)]
        tf = P.shapley_server_submit(srv, H, of)
        # the later requests are admitted while earlier ones are on the device
        act = P.shapley_server_step(srv)
        steps += 1
        overlap = [t for t in running_early if P.shapley_server_poll(srv, t) is None]
        max_active = max(max_active, act)
        log(f"  running when the second wave was submitted: {len(running_early)}, "
            f"info {P.shapley_server_info(srv)}")
        assert running_early and max_active >= 2
        while True:
            act = P.shapley_server_step(srv)
            max_active = max(max_active, act)
            steps += 1
            if act == 0 or steps > 5000:
                break
        stats = [P.shapley_server_poll(srv, t) for t in tickets]
        sf = P.shapley_server_poll(srv, tf)
        assert all(s is not None for s in stats) and sf is not None
        log(f"  server steps {steps} max active {max_active}")
        for k, g in enumerate(gs):
            v = P.shapley_get_value(hs[k])
            a, b = P.shapley_get_policy(hs[k])
            ref = oracle.policy_iteration(g)
            va, aa, ba, _ = solve_gpu(g, **LIMITS)
            err, ma, mb, _ = compare_with_oracle(g, v, a, b, ref, 1e-9)
            alone = np.max(np.abs(v - va)) / np.max(np.abs(va))
            log(f"  request {k} n={g.n} latency {stats[k]['seconds']*1e3:.1f} ms vs-oracle {err:.2e} "
                f"vs-alone {alone:.2e}")
            assert err <= 1e-9 and len(ma) == 0 and len(mb) == 0 and alone <= 1e-12
        ref = oracle.policy_iteration(lv[-1])
        v = P.shapley_get_value(H)
        a, b = P.shapley_get_policy(H)
        err, ma, mb, _ = compare_with_oracle(lv[-1], v, a, b, ref, 1e-9)
        log(f"  famg request vs-oracle {err:.2e} grids {sf['fmg_levels']}")
        assert err <= 1e-9 and len(ma) == 0 and sf["fmg_levels"] == len(lv)
    finally:
        P.shapley_server_destroy(srv)
        for h in hs:
            P.shapley_game_destroy(h)
        P.shapley_game_destroy(H)


def test_reuse_and_forcing_reach_the_same_fixed_point():
    """Hierarchy reuse and inexact solves change the path, not the fixed point."""
    g = configs.c1(points=65)
    ref = oracle.policy_iteration(g)
    a0 = np.zeros(g.n, np.int32)
    for reuse, forcing in ((0.0, 0.0), (0.5, 0.0), (0.05, 0.1)):
        v, a, b, st = solve_gpu(g, alpha0=a0, beta0=a0, reuse_frac=reuse, forcing=forcing, **LIMITS)
        err, ma, mb, _ = compare_with_oracle(g, v, a, b, ref, 1e-9)
        log(f"  reuse {reuse} forcing {forcing}: err {err:.2e} outer {st['outer']} cycles {st['cycles_total']}")
        assert err <= 1e-9 and len(ma) == 0


def test_workspace_reuse_and_release():
    """Solves reuse the workspace kept for a game's stream: repeated solves,
    batches and hierarchies give identical results, and destroying games in
    any order releases the workspace without touching destroyed streams."""
    import torch
    ga, gb = configs.c0(s=17), configs.c1(points=33)
    ha, hb = P.create_from(ga), P.create_from(gb)
    o = P.shapley_default_opts(**LIMITS)
    P.shapley_solve(ha, o)
    v1 = P.shapley_get_value(ha)
    P.shapley_solve(hb, o)
    P.shapley_solve(ha, o)                       # engine reused after another game
    v2 = P.shapley_get_value(ha)
    np.testing.assert_array_equal(v1, v2)
    P.shapley_solve_batch([hb, ha], o)            # cached under hb's stream
    v3 = P.shapley_get_value(ha)
    assert np.max(np.abs(v3 - v1)) <= 1e-12 * np.max(np.abs(v1))
    s = torch.cuda.Stream()
    os_ = P.shapley_default_opts(stream=s.cuda_stream, **LIMITS)  # caller's stream: not kept
    P.shapley_solve(ha, os_)
    np.testing.assert_array_equal(P.shapley_get_value(ha), v1)
    P.shapley_game_destroy(hb)                    # drops the batch engine first
    P.shapley_game_destroy(ha)
    hc = P.create_from(ga)
    P.shapley_solve(hc, o)
    np.testing.assert_array_equal(P.shapley_get_value(hc), v1)
    P.shapley_game_destroy(hc)
    log("  workspace reuse ok")


def test_planted_exact_ties_greedy_and_solve():
    """Copied actions plant exact ties (bit-identical rows) at every state.
    The HIP greedy sweep at random v takes the lowest index attaining each
    extremum, exactly as the oracle's (Sec. 2: argmax/argmin are sets; the
    reading fixes the lowest index); policy iteration reaches the value of the
    game without the copies, and its choices at tied states are extrema."""
    base = configs.c0(s=17)
    g = games.with_copied_action(games.with_copied_action(base, 1, 1, 3), 2, 0, 1)
    h = P.create_from(g)
    try:
        rng = np.random.default_rng(3)
        for k in range(3):
            v = rng.normal(size=g.n) * 0.1
            F, a, b = P.shapley_apply_operator(h, v)
            ao, bo = oracle.greedy(g, v)
            np.testing.assert_allclose(F, oracle.shapley_operator(g, v), rtol=0, atol=1e-13)
            np.testing.assert_array_equal(a, ao)
            np.testing.assert_array_equal(b, bo)
    finally:
        P.shapley_game_destroy(h)
    ref0 = oracle.policy_iteration(base)
    ref = oracle.policy_iteration(g)
    for prec, tol in ((P.SHAPLEY_FP64, 1e-9), (P.SHAPLEY_MIXED, 1e-6)):
        v, a, b, st = solve_gpu(g, precision=prec, **LIMITS)
        err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, tol)
        e0 = np.max(np.abs(v - ref0.v)) / np.max(np.abs(ref0.v))
        log(f"  planted ties prec {prec}: err {err:.2e} vs untied game {e0:.2e} tied {tied.sum()}/{g.n}")
        assert st["converged"] == 1 and err <= tol and e0 <= tol
        assert tied.sum() > g.n // 4
        assert len(ma) == 0 and len(mb) == 0


def test_planted_ties_random_general_game():
    """Random general game with invalid pairs and copied actions (dense path)."""
    base = games.random_game(50, 2, 3, 91, mu=0.9, density=0.2, invalid_frac=0.2)
    g = games.with_copied_action(games.with_copied_action(base, 1, 0, 2), 2, 2, 1)
    ref = oracle.policy_iteration(g)
    v, a, b, st = solve_gpu(g, **LIMITS)
    err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, 1e-9)
    log(f"  random planted ties: err {err:.2e} tied {tied.sum()}/{g.n}")
    assert err <= 1e-9 and len(ma) == 0 and len(mb) == 0 and tied.any()
