"""The tie-aware comparison used by the GPU parity tests, checked on the CPU
with oracle results and planted choices (no GPU calls)."""
import numpy as np

import oracle
from shapley_inputs import games
from tests.gpu_helpers import compare_with_oracle


def _tie_case():
    base = games.random_game(30, 2, 3, 90, mu=0.9, density=0.3)
    g = games.with_copied_action(games.with_copied_action(base, 1, 0, 2), 2, 1, 3)
    ref = oracle.policy_iteration(g)
    return g, ref


def test_identical_result_passes():
    g, ref = _tie_case()
    err, ma, mb, tied = compare_with_oracle(g, ref.v.copy(), ref.alpha.copy(), ref.beta.copy(), ref, 1e-9)
    assert err == 0.0 and len(ma) == 0 and len(mb) == 0
    assert tied.any()


def test_other_extremum_at_a_tie_passes_and_a_wrong_choice_fails():
    g, ref = _tie_case()
    tied = oracle.tied_states(g, ref.v, ref.alpha)
    # MAX's copy (index 2) of action 0 is as good wherever action 0 is chosen
    xs = np.nonzero(tied & (ref.alpha == 0))[0]
    assert len(xs) > 0
    a = ref.alpha.copy()
    a[xs] = 2
    _, ma, mb, _ = compare_with_oracle(g, ref.v, a, ref.beta, ref, 1e-9)
    assert len(ma) == 0 and len(mb) == 0
    # MIN's copy (index 3) of action 1 where MIN plays 1
    ys = np.nonzero(tied & (ref.beta == 1))[0]
    b = ref.beta.copy()
    b[ys] = 3
    _, ma, mb, _ = compare_with_oracle(g, ref.v, ref.alpha, b, ref, 1e-9)
    assert len(ma) == 0 and len(mb) == 0
    # a strictly worse MAX action at a tied state is flagged
    Q, _ = oracle.q_values(g, ref.v)
    inner = np.where(np.isnan(Q), np.inf, Q).min(axis=2)
    bad = a.copy()
    flagged = []
    for x in xs:
        worse = [k for k in range(g.m1) if inner[x, k] < inner[x, 0] - 1e-6]
        if worse:
            bad[x] = worse[0]
            flagged.append(x)
    assert flagged
    _, ma, _, _ = compare_with_oracle(g, ref.v, bad, ref.beta, ref, 1e-9)
    assert set(flagged) <= set(ma.tolist())
    # a value error above the tolerance is reported
    err, _, _, _ = compare_with_oracle(g, ref.v * (1 + 1e-6), ref.alpha, ref.beta, ref, 1e-9)
    assert err > 1e-9
