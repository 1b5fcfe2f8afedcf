"""The kernels of the AMG setup are a speed choice only (Sec. 4.3).

* The extended+i interpolation of coarse levels by four lanes per row forms
  every weight with the wavefront kernel's operations in the same order.
* The row-wise Galerkin product A_{l+1} = R A_l P by a thread per row (rows
  of up to 16 or 32 columns), four lanes per row (32 or 64), a wavefront per
  row or a workgroup per row generates each coarse entry's products in one
  order (R's row, A's row, P's slots) and adds them one after the other from
  zero.

So every level of the hierarchy, and every solve, is the same bit for bit
whichever kernel took which row.  The games are large enough for the
row-wise product (levels of 8192 coarse rows or more): a 2-D five-point
grid, a 3-D seven-point grid and a point cloud whose coarse rows overflow the
thread kernel."""
import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs, games
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

CASES = [("isaacs2d 257 mixed", lambda: configs.c3_game(3, 257, 0.7), P.SHAPLEY_MIXED),
         ("isaacs3d 33 fp64", lambda: configs.c2(s=33), P.SHAPLEY_FP64),
         ("point cloud 2^15 mixed", lambda: games.point_cloud_game(1 << 15, 11), P.SHAPLEY_MIXED)]


def levels_of(h):
    out = []
    n_lev = P.shapley_hierarchy_level(h, 0, sizes_only=True)["levels"]
    for l in range(n_lev):
        d = P.shapley_hierarchy_level(h, l)
        out.append((d["rp"].copy(), d["ci"].copy(), d["a"].copy()))
    return out


@pytest.mark.parametrize("name,make,precision", CASES, ids=[c[0] for c in CASES])
def test_setup_kernel_choice_does_not_change_results(name, make, precision):
    g = make()
    ref = None
    try:
        for cols, interp in ((0, 0), (1, 0), (4, 4), (-1, -1)):
            P.shapley_tune_galerkin(cols)
            P.shapley_tune_interp(interp)
            h = P.create_from(g)
            try:
                st = P.shapley_solve(h, P.shapley_default_opts(precision=precision, max_outer=500, max_inner=500))
                v = P.shapley_get_value(h)
                a, b = P.shapley_get_policy(h)
                lev = levels_of(h)
            finally:
                P.shapley_game_destroy(h)
            log(f"  {name} galerkin {cols} interp {interp}: outer {st['outer']} cycles {st['cycles_total']} "
                f"levels {len(lev)} sizes {[len(x[0]) - 1 for x in lev]} residual {st['residual']:.3e}")
            assert st["converged"] == 1
            if ref is None:
                ref = (v, a, b, st["cycles_total"], lev)
                continue
            assert len(lev) == len(ref[4])
            for l, (x, y) in enumerate(zip(lev, ref[4])):
                for u, w in zip(x, y):
                    np.testing.assert_array_equal(u, w, err_msg=f"level {l}")
            np.testing.assert_array_equal(v, ref[0])
            np.testing.assert_array_equal(a, ref[1])
            np.testing.assert_array_equal(b, ref[2])
            assert st["cycles_total"] == ref[3]
    finally:
        P.shapley_tune_galerkin(-1)
        P.shapley_tune_interp(-1)

