"""The lanes per sparse row of the cycle kernels are a speed choice only
(Sec. 4.3, the multigrid cycle): every row sum is formed in one fixed order
(entry t into partial sum t mod 4, a fixed butterfly over the partial sums),
so a solve gives the same values and policies bit for bit whether the lane
count is tuned per level or forced to 1, 2 or 4 for every level.  The
games cover five-point (2-D) and seven-point (3-D) level-0 stencils and the
long rows of the coarse levels, in FP64 and in FP32 cycles with FP64
refinement."""
import numpy as np
import pytest

import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

CASES = [("isaacs3d 17", lambda: configs.c2(s=17), P.SHAPLEY_FP64),
         ("isaacs3d 17 mixed", lambda: configs.c2(s=17), P.SHAPLEY_MIXED),
         ("isaacs2d 65", lambda: configs.c3_game(1, 65, 2.0), P.SHAPLEY_FP64)]


@pytest.mark.parametrize("name,make,precision", CASES, ids=[c[0] for c in CASES])
def test_lane_count_does_not_change_results(name, make, precision):
    g = make()
    ref = None
    try:
        for lanes in (0, 1, 2, 4):
            P.shapley_tune_lanes(lanes)
            h = P.create_from(g)
            try:
                st = P.shapley_solve(h, P.shapley_default_opts(precision=precision, max_outer=500, max_inner=500))
                v = P.shapley_get_value(h)
                a, b = P.shapley_get_policy(h)
            finally:
                P.shapley_game_destroy(h)
            log(f"  {name} lanes {lanes}: outer {st['outer']} cycles {st['cycles_total']} "
                f"residual {st['residual']:.3e}")
            assert st["converged"] == 1
            if ref is None:
                ref = (v, a, b, st["cycles_total"])
                continue
            np.testing.assert_array_equal(v, ref[0])
            np.testing.assert_array_equal(a, ref[1])
            np.testing.assert_array_equal(b, ref[2])
            assert st["cycles_total"] == ref[3]
    finally:
        P.shapley_tune_lanes(0)
