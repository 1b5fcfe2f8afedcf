"""Helpers shared by the GPU tests: tie-aware comparison against the oracle."""
import sys

import numpy as np

import oracle
import paper_1107_1653_amd as P


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_with_oracle(g, v, alpha, beta, ref, rel_tol, gap=1e-10):
    """Values within rel_tol (sup-norm relative) and policies identical at
    untied states (top-two gap >= `gap` at the oracle's value)."""
    scale = max(np.max(np.abs(ref.v)), 1e-300)
    err = np.max(np.abs(v - ref.v)) / scale
    tied = oracle.tied_states(g, ref.v, ref.alpha, gap)
    mism_a = np.nonzero((alpha != ref.alpha) & ~tied)[0]
    # MIN's choice only matters at MAX's action; compare where alpha agrees
    same_a = alpha == ref.alpha
    mism_b = np.nonzero((beta != ref.beta) & ~tied & same_a)[0]
    return err, mism_a, mism_b, tied


def solve_gpu(game, **opts):
    h = P.create_from(game)
    try:
        o = P.shapley_default_opts(**opts)
        st = P.shapley_solve(h, o)
        v = P.shapley_get_value(h)
        a, b = P.shapley_get_policy(h)
    finally:
        P.shapley_game_destroy(h)
    return v, a, b, st
