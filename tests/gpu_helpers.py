"""Helpers shared by the GPU tests: tie-aware comparison against the oracle."""
import sys

import numpy as np

import oracle
import paper_1107_1653_amd as P


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tie_validity(g, v_ref, alpha, beta, tol):
    """States where the HIP choice is not an extremum within `tol` at the
    oracle's value: MAX's action must attain max_a min_b Q - tol, MIN's action
    min_b Q(x, alpha(x), b) + tol at the HIP's own alpha (argmax and argmin are
    sets, Sec. 2), and both must be valid pairs."""
    Q, _ = oracle.q_values(g, v_ref)
    xs = np.arange(g.n)
    ok_pair = np.isfinite(Q[xs, alpha, beta]) if g.n else np.zeros(0, bool)
    Qb = np.where(np.isnan(Q), np.inf, Q)
    inner = Qb.min(axis=2)
    inner = np.where(np.isinf(inner), -np.inf, inner)
    F = inner.max(axis=1)
    bad_a = ~(inner[xs, alpha] >= F - tol)
    Qa = Qb[xs, alpha, :]
    bad_b = ~(Qa[xs, beta] <= Qa.min(axis=1) + tol)
    return np.nonzero(bad_a | bad_b | ~ok_pair)[0]


def compare_with_oracle(g, v, alpha, beta, ref, rel_tol, gap=1e-10):
    """Values within rel_tol (sup-norm relative); policies identical at untied
    states (top-two gap >= `gap` at the oracle's value); at tied states the HIP
    choice must still attain the extremum to within the gap plus what the value
    difference can move a row (|Q(v) - Q(v*)| <= mu ||v - v*||, rows
    substochastic).  Returns (err, untied alpha mismatches, untied beta
    mismatches, tied mask); a tied state whose choice is not an extremum counts
    as an alpha mismatch."""
    scale = max(np.max(np.abs(ref.v)), 1e-300)
    dv = np.max(np.abs(v - ref.v)) if g.n else 0.0
    err = dv / scale
    tied = oracle.tied_states(g, ref.v, ref.alpha, gap)
    mism_a = np.nonzero((alpha != ref.alpha) & ~tied)[0]
    # MIN's choice only matters at MAX's action; compare where alpha agrees
    same_a = alpha == ref.alpha
    mism_b = np.nonzero((beta != ref.beta) & ~tied & same_a)[0]
    if tied.any():
        bad = tie_validity(g, ref.v, alpha, beta, gap + 2.0 * g.mu * dv)
        bad_tied = np.intersect1d(bad, np.nonzero(tied)[0])
        mism_a = np.union1d(mism_a, bad_tied)
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
