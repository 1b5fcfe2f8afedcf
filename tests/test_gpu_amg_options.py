"""Multigrid options of the inner solve (Sec. 4.3, Algorithm MGcycle; the
paper's own configuration in Sec. 6 uses W(1,1) cycles with a smoother that
relaxes C points before F points): every combination of relaxation and cycle
index reaches the oracle's fixed point, and the number of cycles per linear
system does not grow with the grid (Sec. 6.1: the AMG iteration counts of
Tables Iex1t1-Iex1t6 are the same at every size)."""
import numpy as np
import pytest

import oracle
import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import compare_with_oracle, log, solve_gpu

pytestmark = pytest.mark.gpu

LIMITS = dict(max_outer=500, max_inner=500)
VARIANTS = [
    ("jacobi V(2,2)", dict(smoother=P.SHAPLEY_SMOOTH_JACOBI, gamma=1)),
    ("l1 V(2,2)", dict(smoother=P.SHAPLEY_SMOOTH_L1, gamma=1)),
    ("cf V(1,1)", dict(smoother=P.SHAPLEY_SMOOTH_CF, gamma=1, nu1=1, nu2=1)),
    ("jacobi W(1,1)", dict(smoother=P.SHAPLEY_SMOOTH_JACOBI, gamma=2, nu1=1, nu2=1)),
    ("cf W(1,1)", dict(smoother=P.SHAPLEY_SMOOTH_CF, gamma=2, nu1=1, nu2=1)),
]


@pytest.mark.parametrize("name,amg", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_options_reach_the_fixed_point(name, amg):
    cases = [("isaacs 2-D 33", configs.c0(s=33), None),
             ("obstacle 65", configs.c1(points=65), np.zeros(63 * 63, np.int32)),
             ("isaacs 3-D 17", configs.c2(s=17), None)]
    for what, g, a0 in cases:
        ref = oracle.policy_iteration(g, alpha0=a0, beta0=a0)
        for prec, tol in ((P.SHAPLEY_FP64, 1e-9), (P.SHAPLEY_MIXED, 1e-6)):
            kw = dict(amg, precision=prec, **LIMITS)
            if a0 is not None:
                kw.update(alpha0=a0, beta0=a0)
            v, a, b, st = solve_gpu(g, **kw)
            err, ma, mb, _ = compare_with_oracle(g, v, a, b, ref, tol)
            log(f"  {name} {what} prec {prec}: err {err:.1e} cycles/system "
                f"{st['cycles_total'] / max(st['value_steps'], 1):.1f} levels {st['levels']}")
            assert st["converged"] == 1 and err <= tol and len(ma) == 0 and len(mb) == 0


def cycles_per_system(side, amg):
    """Cycles per linear system of a full AMGpi solve, each system solved to
    an absolute residual of 1e-10 times the largest reward: a reduction that
    does not depend on the grid (the rewards of the normalised scheme scale
    like h^2, Sec. 6.1 eq. Iex1d), as the paper's fixed residual target."""
    g = configs.c3_game(7, side, 1.0)
    h = P.create_from(g)
    try:
        st = P.shapley_solve(h, P.shapley_default_opts(lin_rtol=0.0, lin_atol=1e-10 * float(np.abs(g.r).max()),
                                                       **amg, **LIMITS))
        assert st["converged"] == 1
        return st["cycles_total"] / st["value_steps"], st
    finally:
        P.shapley_game_destroy(h)


@pytest.mark.parametrize("name,amg", [VARIANTS[0], VARIANTS[4]], ids=[VARIANTS[0][0], VARIANTS[4][0]])
def test_cycle_counts_are_grid_independent(name, amg):
    """2-D Isaacs games from 65^2 to 1025^2 grid points (63^2 ... 1023^2
    unknowns): the average number of cycles per linear system stays within
    +-2 of its middle value."""
    counts = []
    for side in (63, 127, 255, 511, 1023):
        c, st = cycles_per_system(side, amg)
        counts.append(c)
        log(f"  {name} side {side}: {c:.2f} cycles per system over {st['value_steps']} systems, "
            f"levels {st['levels']} op complexity {st['op_complexity']:.2f}")
    mid = 0.5 * (max(counts) + min(counts))
    assert max(counts) - mid <= 2.0, counts
