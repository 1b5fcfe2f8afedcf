"""The algebraic multigrid hierarchy (Sec. 4.3) the device builds, read back
through shapley_hierarchy_level and checked against definitions computed
here with scipy.sparse:

* every coarse operator is the Galerkin product A_{l+1} = P_l^T A_l P_l of
  the level above and its prolongation (large levels take the row-wise
  product -- as R A P, or as R (A P) on levels averaging 16 or more entries
  per row --, small ones the dense per-game blocks: all are covered, after
  full setups and after the numeric refreshes of later policy steps);
* P_l has at most pw distinct entries per row, columns inside the next
  level, and the coarse points are injected: every coarse index J is a fine
  row whose only entry is (J, 1);
* level 0 is the operator I - mu P of the policies the hierarchy was last
  built or refreshed from (its row sums are 1 - mu * sum of the transition
  weights, so they lie in [1 - mu, 1]).

The tolerance is rounding only: each product entry is a sum of a few hundred
terms at most, so 1e-12 of the largest coarse entry.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def level_matrices(h):
    first = P.shapley_hierarchy_level(h, 0)
    levels = []
    for l in range(first["levels"]):
        d = P.shapley_hierarchy_level(h, l)
        A = sp.csr_matrix((d["a"], d["ci"], d["rp"]), shape=(d["n"], d["n"]))
        Pm = None
        if d["nc"]:
            rows = np.repeat(np.arange(d["n"]), d["pw"])
            cols = d["pc"].reshape(-1)
            vals = d["pv"].reshape(-1)
            keep = cols >= 0
            assert np.all(cols[keep] < d["nc"])
            Pm = sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(d["n"], d["nc"]))
            # no duplicate column within a row
            assert Pm.nnz == int(keep.sum())
        levels.append((d, A, Pm))
    return levels


def check_hierarchy(h, what):
    levels = level_matrices(h)
    assert len(levels) >= 2, "expected a multilevel hierarchy"
    for l, (d, A, Pm) in enumerate(levels):
        # columns sorted and distinct within each row
        for i in range(0, d["n"], max(1, d["n"] // 200)):
            c = d["ci"][d["rp"][i]:d["rp"][i + 1]]
            assert np.all(np.diff(c) > 0)
        if Pm is None:
            continue
        Ac = levels[l + 1][1]
        # injection of the coarse points: coarse index J is a fine row whose
        # only entry is (J, 1)
        cnt = np.diff(Pm.indptr)
        one = np.nonzero(cnt == 1)[0]
        first = Pm.indptr[one]
        inj = one[Pm.data[first] == 1.0]
        injected = np.zeros(d["nc"], bool)
        injected[Pm.indices[Pm.indptr[inj]]] = True
        assert injected.all(), "every coarse index is an injected fine row"
        G = (Pm.T @ A @ Pm).tocsr()
        scale = max(np.max(np.abs(Ac.data)), 1e-300)
        diff = (G - Ac).tocsr()
        err = np.max(np.abs(diff.data)) / scale if diff.nnz else 0.0
        # every numerically nonzero entry of the product is in the stored pattern
        Gc = G.tocoo()
        big = np.abs(Gc.data) > 1e-14 * scale
        stored = set(zip(*Ac.nonzero()))
        missing = sum((i, j) not in stored for i, j in zip(Gc.row[big], Gc.col[big]))
        log(f"  {what} level {l} -> {l + 1}: n {d['n']} nnz {d['nnz']} nc {d['nc']}, "
            f"|P^T A P - A_c| / max|A_c| = {err:.2e}, missing {missing}")
        assert err <= 1e-12
        assert missing == 0


def test_galerkin_hierarchy_isaacs2d():
    g = configs.c3_game(0, 129, 1.0)
    h = P.create_from(g)
    try:
        st = P.shapley_solve(h, P.shapley_default_opts(max_outer=500, max_inner=500))
        assert st["converged"] == 1
        check_hierarchy(h, "isaacs2d 129")
        A0 = level_matrices(h)[0][1]
        rs = np.asarray(A0.sum(axis=1)).ravel()
        assert np.all(rs >= 1.0 - g.mu - 1e-12) and np.all(rs <= 1.0 + 1e-12)
    finally:
        P.shapley_game_destroy(h)


def test_galerkin_hierarchy_isaacs3d():
    g = configs.c2(s=17)
    h = P.create_from(g)
    try:
        st = P.shapley_solve(h, P.shapley_default_opts(max_outer=500, max_inner=500,
                                                       precision=P.SHAPLEY_MIXED))
        assert st["converged"] == 1
        check_hierarchy(h, "isaacs3d 17")
    finally:
        P.shapley_game_destroy(h)


def test_galerkin_hierarchy_isaacs3d_long_rows():
    # 33^3: the coarse levels above the dense blocks average more than 16
    # entries per row and take R (A P)
    g = configs.c2(s=33)
    h = P.create_from(g)
    try:
        st = P.shapley_solve(h, P.shapley_default_opts(max_outer=500, max_inner=500, forcing=0.1, reuse_frac=0.5))
        assert st["converged"] == 1
        log(f"  isaacs3d 33: full setups {st['setups_full']} refreshes {st['setups_refresh']}")
        check_hierarchy(h, "isaacs3d 33")
    finally:
        P.shapley_game_destroy(h)


def test_galerkin_hierarchy_obstacle_famg():
    levels = configs.c1_levels(points=129, coarsest_points=33)
    H = P.shapley_game_create_hierarchy([P.create_from(x) for x in levels])
    try:
        a0 = np.zeros(levels[0].n, np.int32)
        st = P.shapley_solve(H, P.shapley_default_opts(method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0,
                                                       max_outer=500, max_inner=500))
        assert st["converged"] == 1
        check_hierarchy(H, "obstacle 129 FAMGpi")
    finally:
        P.shapley_game_destroy(H)


def test_hierarchy_inspection_errors():
    g = configs.c0(s=9)
    h = P.create_from(g)
    try:
        with pytest.raises(P.ShapleyError):  # nothing solved yet on this stream
            P.shapley_hierarchy_level(h, 0)
        P.shapley_solve(h, P.shapley_default_opts())
        n_lev = P.shapley_hierarchy_level(h, 0)["levels"]
        with pytest.raises(P.ShapleyError):
            P.shapley_hierarchy_level(h, n_lev)
    finally:
        P.shapley_game_destroy(h)
