"""The allocation-free entry point (shapley_apply_operator_noalloc) through the
C ABI: device-resident arguments, reductions in the library's fixed device
array, results equal to shapley_apply_operator's; consecutive calls on games
of decreasing size reuse the same array."""
import ctypes as C

import numpy as np
import pytest

import oracle
import paper_1107_1653_amd as P
from shapley_inputs import configs, games
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


def call_noalloc(h, v_host):
    import torch
    n = len(v_host)
    v = torch.from_numpy(np.ascontiguousarray(v_host)).cuda()
    F = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    a = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    b = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    res = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    P.shapley_apply_operator_noalloc(h, v, F, a, b, res)
    torch.cuda.synchronize()
    return F.cpu().numpy(), a.cpu().numpy(), b.cpu().numpy(), res.cpu().numpy()


def test_noalloc_matches_apply_operator_on_consecutive_calls():
    cases = [("isaacs 33^2", configs.c0(s=33)), ("isaacs 17^2 (smaller)", configs.c0(s=17)),
             ("random with invalid pairs (smaller)", games.random_game(50, 3, 3, 77, mu=0.9, density=0.2,
                                                                      invalid_frac=0.2))]
    rng = np.random.default_rng(11)
    for what, g in cases:
        h = P.create_from(g)
        try:
            for rep in range(2):
                v = rng.normal(size=g.n) * 0.1
                F, a, b, res = call_noalloc(h, v)
                F0, a0, b0 = P.shapley_apply_operator(h, v)
                np.testing.assert_array_equal(F, F0)
                np.testing.assert_array_equal(a, a0)
                np.testing.assert_array_equal(b, b0)
                ao, bo = oracle.greedy(g, v)
                np.testing.assert_array_equal(a, ao)
                np.testing.assert_array_equal(b, bo)
                d = F - v
                assert res[0] == np.max(np.abs(d))
                assert res[1] == pytest.approx(np.sum(d * d), rel=1e-12)
                log(f"  {what} call {rep}: n={g.n}, max |F(v) - v| {res[0]:.3e}")
        finally:
            P.shapley_game_destroy(h)


def test_noalloc_rejects_missing_arguments():
    g = configs.c0(s=9)
    h = P.create_from(g)
    try:
        rc = P.lib().shapley_apply_operator_noalloc(h, None, None, None, None, None, None)
        assert rc == P.SHAPLEY_EINVAL and "null" in P.shapley_last_error()
    finally:
        P.shapley_game_destroy(h)
