"""Every SHAPLEY_EINVAL condition of the boundary is driven through the C ABI
on the host, where it is detected before any device call: bad sizes, w < 0,
row sum > 1 + 1e-12, mu outside (0, 1], NaN/Inf, empty action set, bad
options, bad blocks for the coarsest-level inverse.  Inputs that pass the checks reach the device (SHAPLEY_EDEVICE
without a GPU), which shows the checks are not too strict."""
import ctypes as C
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1107_1653_amd", "libshapley.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def small_game():
    from shapley_inputs import games
    return games.random_game(6, 2, 2, 3, mu=0.9, density=0.5)


def create(P, g, **kw):
    """rc and message of shapley_game_create with fields of g overridden."""
    a = dict(n=g.n, m1=g.m1, m2=g.m2, row_ptr=g.row_ptr.copy(), col=g.col.copy(), w=g.w.copy(),
             r=g.r.copy(), mu=g.mu, valid=None if g.valid is None else g.valid.copy(), grid=None, flags=0)
    a.update(kw)
    ptr = lambda x, t: None if x is None else np.ascontiguousarray(x, dtype=t).ctypes.data_as(C.c_void_p)
    keep = [np.ascontiguousarray(a[k]) for k in ("row_ptr", "col", "w", "r") if a[k] is not None]
    gp = None
    if a["grid"] is not None:
        gs = P.shapley_grid()
        gs.dim, gs.s = a["grid"]
        gp = C.byref(gs)
    h = C.c_void_p()
    rc = P.lib().shapley_game_create(C.byref(h), int(a["n"]), int(a["m1"]), int(a["m2"]),
                                     ptr(a["row_ptr"], np.int64), ptr(a["col"], np.int32),
                                     ptr(a["w"], np.float64), ptr(a["r"], np.float64), float(a["mu"]),
                                     ptr(a["valid"], np.uint8), gp, int(a["flags"]), None)
    del keep
    if rc == P.SHAPLEY_OK:
        P.shapley_game_destroy(h)
    return rc, P.shapley_last_error()


@pytest.fixture(scope="module")
def P():
    import paper_1107_1653_amd as P
    P.lib()
    return P


def expect_einval(P, g, needle, **kw):
    rc, msg = create(P, g, **kw)
    assert rc == P.SHAPLEY_EINVAL, (rc, msg)
    assert needle in msg, msg


def test_sizes(P):
    g = small_game()
    expect_einval(P, g, "positive", n=0)
    expect_einval(P, g, "positive", m1=0)
    expect_einval(P, g, "positive", m2=-1)
    expect_einval(P, g, "256", m1=17, m2=16)
    expect_einval(P, g, "2^31", n=1 << 28, m1=4, m2=4)
    expect_einval(P, g, "unsupported flags", flags=7)
    expect_einval(P, g, "null input", r=None)


def test_row_pointer_and_columns(P):
    g = small_game()
    rp = g.row_ptr.copy(); rp[0] = 1
    expect_einval(P, g, "row_ptr[0]", row_ptr=rp)
    rp = g.row_ptr.copy(); rp[3] = rp[2] - 1
    expect_einval(P, g, "non-decreasing", row_ptr=rp)
    rp = g.row_ptr.copy(); rp[2] = rp[-1] + 5
    expect_einval(P, g, "non-decreasing", row_ptr=rp)
    for bad in (-1, g.n):
        c = g.col.copy(); c[4] = bad
        expect_einval(P, g, "column index", col=c)


@pytest.mark.parametrize("bad", [-1e-3, math.nan, math.inf])
def test_weights(P, bad):
    g = small_game()
    w = g.w.copy(); w[2] = bad
    expect_einval(P, g, "weights must be finite", w=w)


def test_row_sum(P):
    g = small_game()
    # one row scaled to sum exactly 1 + 2e-12: rejected; 1 + 5e-13: accepted
    i = 5
    a, b = g.row_ptr[i], g.row_ptr[i + 1]
    for excess, ok in ((2e-12, False), (5e-13, True)):
        w = g.w.copy()
        w[a:b] = w[a:b] / w[a:b].sum() * (1.0 + excess)
        assert (w[a:b].sum() > 1.0 + 1e-12) == (not ok)
        rc, msg = create(P, g, w=w)
        if ok:
            assert rc in (P.SHAPLEY_OK, P.SHAPLEY_EDEVICE), msg   # EDEVICE: no GPU here
        else:
            assert rc == P.SHAPLEY_EINVAL and "row sum" in msg


@pytest.mark.parametrize("mu", [0.0, -0.5, 1.5, math.nan, math.inf])
def test_discount(P, mu):
    expect_einval(P, small_game(), "mu must lie", mu=mu)


@pytest.mark.parametrize("bad", [math.nan, math.inf, -math.inf])
def test_rewards(P, bad):
    g = small_game()
    r = g.r.copy(); r[7] = bad
    expect_einval(P, g, "rewards must be finite", r=r)


def test_empty_action_set(P):
    g = small_game()
    v = np.ones(g.nrows, np.uint8)
    v[2 * 4:3 * 4] = 0      # state 2: no valid pair
    expect_einval(P, g, "empty action set", valid=v)
    v[2 * 4 + 3] = 1        # one valid pair is enough
    rc, msg = create(P, g, valid=v)
    assert rc in (P.SHAPLEY_OK, P.SHAPLEY_EDEVICE), msg


def test_grid_description(P):
    g = small_game()
    expect_einval(P, g, "s^dim", grid=(2, 3))
    expect_einval(P, g, "dim in 1..3", grid=(4, 1))


def test_valid_input_reaches_the_device(P):
    rc, msg = create(P, small_game())
    assert rc in (P.SHAPLEY_OK, P.SHAPLEY_EDEVICE), msg


BAD_OPTS = [("precision", 5, "precision"), ("method", 2, "method"), ("max_outer", 0, "limits"),
            ("max_inner", 0, "limits"), ("max_cycles", 0, "limits"), ("nu1", 0, "nu1"), ("nu2", -1, "nu2"),
            ("omega", 2.0, "omega"), ("omega", 0.0, "omega"), ("coarse_max", 0, "coarse_max"),
            ("coarse_max", 5000, "coarse_max"), ("max_levels", 0, "max_levels"), ("lin_rtol", -1.0, "tolerances"),
            ("tie_rtol", -1e-12, "tolerances"), ("c_fmg", 0.0, "c_fmg"), ("reuse_frac", 1.5, "reuse_frac"),
            ("forcing", 1.0, "forcing"), ("eps", -1.0, "eps"), ("eps", math.nan, "eps"),
            ("smoother", 7, "smoother"), ("gamma", 3, "gamma"), ("graph", 2, "graph"),
            ("theta", math.nan, "finite")]


@pytest.mark.parametrize("field,value,needle", BAD_OPTS)
def test_solve_options(P, field, value, needle):
    """Options are checked before the handle is looked at: a null handle with
    bad options is reported as bad options."""
    o = P.shapley_default_opts()
    setattr(o, field, value)
    rc = P.lib().shapley_solve(None, C.byref(o), None)
    msg = P.shapley_last_error()
    assert rc == P.SHAPLEY_EINVAL and needle in msg, (rc, msg)
    rc = P.lib().shapley_solve_batch(None, 0, C.byref(o), None)
    assert rc == P.SHAPLEY_EINVAL and needle in P.shapley_last_error()
    # the defaults pass the option checks (then the null handle is reported)
    rc = P.lib().shapley_solve(None, None, None)
    assert rc == P.SHAPLEY_EINVAL and "null game" in P.shapley_last_error()


def test_server_arguments(P):
    h = C.c_void_p()
    assert P.lib().shapley_server_create(C.byref(h), 0, None) == P.SHAPLEY_EINVAL
    assert P.lib().shapley_server_create(None, 1 << 30, None) == P.SHAPLEY_EINVAL
    t = C.c_uint64()
    assert P.lib().shapley_server_submit(None, None, None, C.byref(t)) == P.SHAPLEY_EINVAL
    assert P.lib().shapley_server_step(None, None) == P.SHAPLEY_EINVAL
    assert P.lib().shapley_server_poll(None, 1, None) == P.SHAPLEY_EINVAL


def test_coarse_inverse_arguments(P):
    assert P.shapley_coarse_inverse([]) == []
    for bad in ([np.zeros((1025, 1025))], [np.array([[1.0, np.nan], [0.0, 1.0]])],
                [np.eye(3), np.array([[np.inf]])]):
        with pytest.raises(P.ShapleyError) as e:
            P.shapley_coarse_inverse(bad)
        assert e.value.code == P.SHAPLEY_EINVAL
    one = (C.c_double * 1)(1.0)
    size0 = (C.c_int32 * 1)(0)
    assert P.lib().shapley_coarse_inverse(one, size0, 1, one) == P.SHAPLEY_EINVAL
    assert P.lib().shapley_coarse_inverse(None, None, -1, None) == P.SHAPLEY_EINVAL
    assert P.lib().shapley_coarse_inverse(None, size0, 1, one) == P.SHAPLEY_EINVAL
    for bad in (1, 4, -2):
        assert P.lib().shapley_tune_dense(bad) == P.SHAPLEY_EINVAL
