"""The C ABI on the GPU: games created from device memory, error paths that
need a device (device-side input checks, warm starts, iteration limits,
budget), and the request loop's options, overlap and failure isolation."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_1107_1653_amd as P
from shapley_inputs import configs, games
from tests.gpu_helpers import compare_with_oracle, log, solve_gpu

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)


def shuffled_rows(g, seed):
    """The same game with the entries of every row in a random order."""
    rng = np.random.default_rng(seed)
    col, w = g.col.copy(), g.w.copy()
    for i in range(g.nrows):
        a, b = g.row_ptr[i], g.row_ptr[i + 1]
        p = rng.permutation(b - a)
        col[a:b] = g.col[a:b][p]
        w[a:b] = g.w[a:b][p]
    return games.Game(g.n, g.m1, g.m2, g.row_ptr, col, w, g.r, g.mu, g.valid, g.grid, g.meta)


def solve_handle(h, **opts):
    st = P.shapley_solve(h, P.shapley_default_opts(**opts))
    return P.shapley_get_value(h), P.shapley_get_policy(h), st


@pytest.mark.parametrize("which", ["isaacs", "random_valid", "two_stopper_bvals"])
def test_device_pointer_create_matches_host_create(which):
    """SHAPLEY_DEVICE_PTRS: arrays handed over as torch device tensors give
    the same game as host arrays -- the solves agree bit for bit (rows given
    unsorted are sorted on the device as on the host)."""
    g = {"isaacs": lambda: configs.c0(s=17),
         "random_valid": lambda: shuffled_rows(games.random_game(60, 3, 2, 5, mu=0.9, density=0.2,
                                                                 invalid_frac=0.2), 1),
         "two_stopper_bvals": lambda: games.two_stopper_game(129)}[which]()
    log(f"device create {which} n={g.n}")
    hh = P.create_from(g)
    hd = P.create_from(g, device=True)
    try:
        assert P.shapley_game_bytes(hh) == P.shapley_game_bytes(hd)
        for prec in (P.SHAPLEY_FP64, P.SHAPLEY_MIXED):
            vh, (ah, bh), sh = solve_handle(hh, precision=prec, **LIMITS)
            vd, (ad, bd), sd = solve_handle(hd, precision=prec, **LIMITS)
            np.testing.assert_array_equal(vh, vd)
            np.testing.assert_array_equal(ah, ad)
            np.testing.assert_array_equal(bh, bd)
            assert sh["cycles_total"] == sd["cycles_total"] and sh["outer"] == sd["outer"]
        ref = oracle.policy_iteration(g)
        err, ma, mb, _ = compare_with_oracle(g, vd, ad, bd, ref, 1e-6)
        assert err <= 1e-6 and len(ma) == 0 and len(mb) == 0
    finally:
        P.shapley_game_destroy(hh)
        P.shapley_game_destroy(hd)


def test_device_pointer_create_rejects_bad_inputs():
    """The device-side check reports the same conditions as the host one."""
    import torch
    g = games.random_game(20, 2, 2, 8, mu=0.9, density=0.3)

    def try_create(**kw):
        a = dict(row_ptr=g.row_ptr.copy(), col=g.col.copy(), w=g.w.copy(), r=g.r.copy(), valid=None, mu=g.mu)
        a.update(kw)
        t = lambda x, dt: None if x is None else torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).cuda()
        args = [t(a["row_ptr"], np.int64), t(a["col"], np.int32), t(a["w"], np.float64), t(a["r"], np.float64)]
        torch.cuda.synchronize()
        try:
            h = P.shapley_game_create(g.n, g.m1, g.m2, *args, a["mu"], t(a["valid"], np.uint8), None,
                                      P.SHAPLEY_DEVICE_PTRS)
        except P.ShapleyError as e:
            return e.code, str(e)
        P.shapley_game_destroy(h)
        return 0, ""

    cases = []
    w = g.w.copy(); w[3] = -0.1; cases.append(("weights must be finite", dict(w=w)))
    w = g.w.copy(); w[5] = np.nan; cases.append(("weights must be finite", dict(w=w)))
    c = g.col.copy(); c[2] = g.n; cases.append(("column index", dict(col=c)))
    rp = g.row_ptr.copy(); rp[4] = rp[3] - 1; cases.append(("non-decreasing", dict(row_ptr=rp)))
    r = g.r.copy(); r[1] = np.inf; cases.append(("rewards must be finite", dict(r=r)))
    w = g.w.copy(); i = 6; a, b = g.row_ptr[i], g.row_ptr[i + 1]; w[a:b] *= 1.2 / w[a:b].sum()
    cases.append(("row sum", dict(w=w)))
    v = np.ones(g.nrows, np.uint8); v[4:8] = 0; cases.append(("empty action set", dict(valid=v)))
    for needle, kw in cases:
        rc, msg = try_create(**kw)
        log(f"  device check {needle}: rc {rc}")
        assert rc == P.SHAPLEY_EINVAL and needle in msg, msg
    assert try_create()[0] == 0


def test_warm_start_must_be_valid():
    """alpha0 naming an unavailable action, or an invalid (alpha0, beta0) pair,
    is SHAPLEY_EINVAL before the solve changes anything."""
    base = games.random_game(30, 3, 2, 12, mu=0.9, density=0.3)
    valid = np.ones((30, 3, 2), np.uint8)
    valid[4, 2, :] = 0          # state 4: action 2 unavailable
    valid[7, 1, 0] = 0          # state 7: pair (1, 0) invalid
    g = games.Game(base.n, 3, 2, base.row_ptr, base.col, base.w, base.r, base.mu, valid.reshape(-1))
    h = P.create_from(g)
    try:
        P.shapley_solve(h, P.shapley_default_opts(**LIMITS))
        v_before = P.shapley_get_value(h)
        a0 = np.zeros(30, np.int32)
        a0[4] = 2
        with pytest.raises(P.ShapleyError) as e:
            P.shapley_solve(h, P.shapley_default_opts(alpha0=a0, **LIMITS))
        assert e.value.code == P.SHAPLEY_EINVAL and "no valid b" in str(e.value)
        a0[4] = 0
        a0[7] = 1
        b0 = np.zeros(30, np.int32)
        with pytest.raises(P.ShapleyError) as e:
            P.shapley_solve(h, P.shapley_default_opts(alpha0=a0, beta0=b0, **LIMITS))
        assert e.value.code == P.SHAPLEY_EINVAL and "valid pair" in str(e.value)
        np.testing.assert_array_equal(P.shapley_get_value(h), v_before)
        b0[7] = 1
        st = P.shapley_solve(h, P.shapley_default_opts(alpha0=a0, beta0=b0, **LIMITS))
        assert st["converged"] == 1
        ref = oracle.policy_iteration(g)
        err, ma, mb, _ = compare_with_oracle(g, P.shapley_get_value(h), *P.shapley_get_policy(h), ref, 1e-9)
        assert err <= 1e-9 and len(ma) == 0
        # the request loop checks the same at submission
        srv = P.shapley_server_create(1 << 34)
        try:
            a0[4] = 2
            with pytest.raises(P.ShapleyError) as e:
                P.shapley_server_submit(srv, h, P.shapley_default_opts(alpha0=a0, **LIMITS))
            assert e.value.code == P.SHAPLEY_EINVAL
        finally:
            P.shapley_server_destroy(srv)
    finally:
        P.shapley_game_destroy(h)


def test_iteration_limit_returns_enoconv_with_readable_results():
    g = configs.c0(s=17)
    h = P.create_from(g)
    try:
        st = P.shapley_solve(h, P.shapley_default_opts(max_outer=1, max_inner=500), allow_noconv=True)
        assert st["rc"] == P.SHAPLEY_ENOCONV and st["converged"] == 0 and st["outer"] == 1
        assert "iteration limit" in P.shapley_last_error()
        v = P.shapley_get_value(h)
        a, b = P.shapley_get_policy(h)
        assert np.all(np.isfinite(v)) and st["residual"] > 0
        # the partial result is a valid warm start: the solve finishes from it
        st2 = P.shapley_solve(h, P.shapley_default_opts(alpha0=a, beta0=b, v0=v, **LIMITS))
        ref = oracle.policy_iteration(g)
        err, ma, mb, _ = compare_with_oracle(g, P.shapley_get_value(h), *P.shapley_get_policy(h), ref, 1e-9)
        log(f"  enoconv after 1 outer, residual {st['residual']:.2e}; resumed: outer {st2['outer']} err {err:.1e}")
        assert st2["converged"] == 1 and err <= 1e-9 and len(ma) == 0
        # MIN's loop cut at one step: either converged (residual test) or ENOCONV, never a false fixed point
        st3 = P.shapley_solve(h, P.shapley_default_opts(max_outer=500, max_inner=1), allow_noconv=True)
        if st3["rc"] == P.SHAPLEY_OK:
            assert st3["converged"] == 1
            F, _, _ = P.shapley_apply_operator(h, P.shapley_get_value(h))
            assert np.max(np.abs(F - P.shapley_get_value(h))) <= 1e-9 * np.max(np.abs(ref.v))
        else:
            assert st3["rc"] == P.SHAPLEY_ENOCONV and st3["converged"] == 0
    finally:
        P.shapley_game_destroy(h)


def test_request_above_the_whole_budget_is_enomem():
    g = configs.c0(s=33)
    h = P.create_from(g)
    srv = P.shapley_server_create(P.shapley_game_bytes(h))   # the game alone, no room to solve
    try:
        with pytest.raises(P.ShapleyError) as e:
            P.shapley_server_submit(srv, h, P.shapley_default_opts(**LIMITS))
        assert e.value.code == P.SHAPLEY_ENOMEM
        assert P.shapley_server_info(srv)["queued"] == 0
    finally:
        P.shapley_server_destroy(srv)
        P.shapley_game_destroy(h)


def test_server_mixed_options_overlap_and_failure_isolation():
    """Requests with different precisions and tie tolerances each get their
    own solve (the result alone); a request admitted while another is on the
    device runs beside it (two cohorts active); a request whose solve fails
    (coarsest block above the dense limit with max_levels = 1) completes with
    its error and releases its budget while the others finish."""
    gs = [configs.c4_game(0, 33, 2.0, 2101), configs.c4_game(0, 41, 0.5, 2102), configs.c4_game(0, 29, 5.0, 2103)]
    opts = [dict(precision=P.SHAPLEY_FP64), dict(precision=P.SHAPLEY_MIXED), dict(precision=P.SHAPLEY_FP64,
                                                                                   tie_rtol=1e-10)]
    hs = [P.create_from(g) for g in gs]
    bad = P.create_from(configs.c0(s=33))
    srv = P.shapley_server_create(200 * 10 ** 9)
    try:
        t0 = P.shapley_server_submit(srv, hs[0], P.shapley_default_opts(**opts[0], **LIMITS))
        assert P.shapley_server_step(srv) == 1
        assert P.shapley_server_poll(srv, t0) is None         # still running
        t1 = P.shapley_server_submit(srv, hs[1], P.shapley_default_opts(**opts[1], **LIMITS))
        t2 = P.shapley_server_submit(srv, hs[2], P.shapley_default_opts(**opts[2], **LIMITS))
        tb = P.shapley_server_submit(srv, bad, P.shapley_default_opts(max_levels=1, **LIMITS))
        act = P.shapley_server_step(srv)
        info = P.shapley_server_info(srv)
        log(f"  after the second step: active {act}, {info}")
        assert P.shapley_server_poll(srv, t0) is None or act >= 2
        assert info["cohorts"] >= 2                            # admitted beside the running request
        steps = 2
        while P.shapley_server_step(srv) > 0:
            steps += 1
            assert steps < 5000
        sb = P.shapley_server_poll(srv, tb)        # ENOCONV is returned with stats, not raised
        assert sb["rc"] == P.SHAPLEY_ENOCONV and sb["converged"] == 0
        assert "dense" in P.shapley_last_error()
        info = P.shapley_server_info(srv)
        assert info["active"] == 0 and info["budget_used"] == 0
        for k, t in enumerate((t0, t1, t2)):
            st = P.shapley_server_poll(srv, t)
            v = P.shapley_get_value(hs[k])
            a, b = P.shapley_get_policy(hs[k])
            va, aa, ba, _ = solve_gpu(gs[k], **opts[k], **LIMITS)
            alone = np.max(np.abs(v - va)) / np.max(np.abs(va))
            ref = oracle.policy_iteration(gs[k])
            tol = 1e-6 if opts[k]["precision"] == P.SHAPLEY_MIXED else 1e-9
            err, ma, mb, _ = compare_with_oracle(gs[k], v, a, b, ref, tol)
            log(f"  request {k} {opts[k]}: vs alone {alone:.1e}, vs oracle {err:.1e}, outer {st['outer']}")
            assert st["converged"] == 1 and alone <= 1e-12 and err <= tol and len(ma) == 0 and len(mb) == 0
            np.testing.assert_array_equal(a, aa)
    finally:
        P.shapley_server_destroy(srv)
        for h in hs:
            P.shapley_game_destroy(h)
        P.shapley_game_destroy(bad)
