"""The exact solve on the coarsest level of the multigrid cycle (Algorithm
MGcycle, Sec. 4.3): each coarsest block is inverted once per setup.

Blocks of at most 64 unknowns take the FP64 matrix-core kernel (a blocked
Gauss-Jordan sweep over panels of 16 columns with partial pivoting) or, with
shapley_tune_dense(0), the register Gauss-Jordan kernel; larger blocks take the
Gauss-Jordan kernels of 96 and 1024 unknowns.  The inverse is a plain
definition, so LAPACK's (numpy.linalg.inv) is the reference, to the rounding
that the block's condition number allows; blocks with exact inverses
(permutations, diagonal powers of two, triangular 0/1 patterns) must come out
exact; singular blocks are reported."""
import numpy as np
import pytest

import oracle
import paper_1107_1653_amd as P
from shapley_inputs import configs
from tests.gpu_helpers import compare_with_oracle, log

pytestmark = pytest.mark.gpu

KERNELS = [(-1, "matrix cores"), (0, "register Gauss-Jordan")]


def _blocks(sizes, kind, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        if kind == "gaussian":
            A = rng.standard_normal((n, n))
        elif kind == "policy":  # I - mu W, W substochastic: the coarse operators' family
            W = np.abs(rng.standard_normal((n, n))) * (rng.random((n, n)) < 0.3)
            W /= np.maximum(W.sum(axis=1, keepdims=True), 1e-300)
            A = np.eye(n) - 0.95 * W
        else:  # "pivoting": a zero diagonal (n > 1), so that every step has to exchange rows
            A = rng.standard_normal((n, n))
            if n > 1:
                A[np.arange(n), np.arange(n)] = 0.0
        out.append(A)
    return out


@pytest.mark.parametrize("kernel,kname", KERNELS, ids=[k[1] for k in KERNELS])
@pytest.mark.parametrize("kind", ["gaussian", "policy", "pivoting"])
def test_coarse_inverse_matches_lapack(kernel, kname, kind):
    sizes = list(range(1, 65)) + [17, 48, 63]  # every padded width, ragged tails
    blocks = _blocks(sizes, kind, 7 + len(kind))
    try:
        P.shapley_tune_dense(kernel)
        inv = P.shapley_coarse_inverse(blocks)
    finally:
        P.shapley_tune_dense(-1)
    worst = 0.0
    for A, X in zip(blocks, inv):
        n = A.shape[0]
        ref = np.linalg.inv(A)
        cond = np.linalg.cond(A, 1)
        err = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
        # forward error of a backward-stable inverse: a modest multiple of n u cond(A)
        bound = 64.0 * n * np.finfo(float).eps * max(cond, 1.0)
        worst = max(worst, err / bound)
        assert err <= bound, f"n={n} err={err:.3e} cond={cond:.3e}"
        assert np.max(np.abs(X @ A - np.eye(n))) <= bound * max(1.0, np.max(np.abs(A)) * np.max(np.abs(ref)))
    log(f"  {kname} {kind}: worst error / bound {worst:.3e}")


@pytest.mark.parametrize("kernel,kname", KERNELS, ids=[k[1] for k in KERNELS])
def test_coarse_inverse_exact_cases(kernel, kname):
    rng = np.random.default_rng(3)
    blocks, refs = [], []
    for n in (1, 5, 16, 31, 64):
        Pm = np.eye(n)[rng.permutation(n)]
        blocks.append(Pm)
        refs.append(Pm.T.copy())
        d = 2.0 ** rng.integers(-6, 7, n).astype(float) * rng.choice([-1.0, 1.0], n)
        blocks.append(np.diag(d))
        refs.append(np.diag(1.0 / d))
        U = np.eye(n) + np.diag(np.ones(n - 1), 1)  # inverse: alternating signs above the diagonal
        blocks.append(U)
        i, j = np.indices((n, n))
        refs.append(np.where(j >= i, (-1.0) ** (j - i), 0.0))
    try:
        P.shapley_tune_dense(kernel)
        inv = P.shapley_coarse_inverse(blocks)
    finally:
        P.shapley_tune_dense(-1)
    for X, R in zip(inv, refs):
        np.testing.assert_array_equal(X, R)


@pytest.mark.parametrize("kernel,kname", KERNELS, ids=[k[1] for k in KERNELS])
def test_coarse_inverse_reports_singular_blocks(kernel, kname):
    good = _blocks([20], "policy", 1)[0]
    for n in (3, 40, 64):
        S = _blocks([n], "gaussian", n)[0]
        S[:, n // 2] = 0.0  # a zero column: no pivot left at that step
        try:
            P.shapley_tune_dense(kernel)
            with pytest.raises(P.ShapleyError) as e:
                P.shapley_coarse_inverse([good, S])
        finally:
            P.shapley_tune_dense(-1)
        assert e.value.code == P.SHAPLEY_EDEVICE


def test_larger_blocks_take_the_gauss_jordan_kernels():
    sizes = [65, 96, 97, 200, 5]
    blocks = _blocks(sizes, "policy", 11)
    inv = P.shapley_coarse_inverse(blocks)
    for A, X in zip(blocks, inv):
        n = A.shape[0]
        ref = np.linalg.inv(A)
        bound = 64.0 * n * np.finfo(float).eps * max(np.linalg.cond(A, 1), 1.0)
        assert np.max(np.abs(X - ref)) / np.max(np.abs(ref)) <= bound


@pytest.mark.parametrize("precision", [P.SHAPLEY_FP64, P.SHAPLEY_MIXED], ids=["fp64", "mixed"])
def test_solves_with_either_coarse_kernel_match_the_oracle(precision):
    g = configs.c0()
    ref = oracle.policy_iteration(g)
    tol = 1e-9 if precision == P.SHAPLEY_FP64 else 1e-6
    for kernel, kname in KERNELS:
        try:
            P.shapley_tune_dense(kernel)
            h = P.create_from(g)
            try:
                st = P.shapley_solve(h, P.shapley_default_opts(precision=precision, coarse_max=64))
                v = P.shapley_get_value(h)
                a, b = P.shapley_get_policy(h)
            finally:
                P.shapley_game_destroy(h)
        finally:
            P.shapley_tune_dense(-1)
        err, ma, mb, tied = compare_with_oracle(g, v, a, b, ref, tol)
        log(f"  {kname}: outer {st['outer']} cycles {st['cycles_total']} rel err {err:.2e}")
        assert st["converged"] == 1
        assert err <= tol and len(ma) == 0 and len(mb) == 0
