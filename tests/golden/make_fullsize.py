"""Writes the full-size parity fixtures from the oracle alone.

    python tests/golden/make_fullsize.py obstacle   # -> obstacle_1025.json
    python tests/golden/make_fullsize.py isaacs3d   # -> isaacs3d_129.json, isaacs3d_129_full.npz

Each fixture holds the oracle's fixed point (value, strategies of both
players and a tie flag) at a seeded sample of states of one benchmark
workload, so that a GPU test can compare the device solution at those states
without re-running the oracle:

* obstacle_1025.json -- the obstacle problem (variational inequality of
  Sec. 6.1 with a stop action), 1025 points per side including the boundary,
  solved by the oracle's FAMGpi (Sec. 5.2) on the nested grids 33 ... 1025
  with c = 1e-2 and eps = 0 on the finest grid (run until no policy
  improves).
* isaacs3d_129.json -- the 3-D Isaacs game, 129 interior points per side,
  oracle policy iteration (Sec. 4.2) from the default start with the Krylov
  policy evaluation (the sparse LU does not fit in memory at this size),
  eps = 0.  isaacs3d_129_full.npz holds the same fixed point at every state
  (the oracle takes minutes here, too long to run beside a GPU test).

Only the seeded generators and `oracle` are used.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from shapley_inputs import configs  # noqa: E402

SAMPLES = 1024
BOUNDARY_SAMPLES = 256


def sample_states(n, alpha, shape, seed):
    """Seeded uniform sample plus states at which MAX's strategy differs from
    a grid neighbour's (the free boundary, where a wrong decision shows)."""
    rng = np.random.default_rng(seed)
    uni = rng.choice(n, size=min(SAMPLES, n), replace=False)
    a = alpha.reshape(shape)
    edge = np.zeros(shape, dtype=bool)
    for ax in range(len(shape)):
        d = np.diff(a, axis=ax) != 0
        lo = [slice(None)] * len(shape)
        hi = [slice(None)] * len(shape)
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        edge[tuple(lo)] |= d
        edge[tuple(hi)] |= d
    cand = np.flatnonzero(edge.reshape(-1))
    if len(cand):
        cand = rng.choice(cand, size=min(BOUNDARY_SAMPLES, len(cand)), replace=False)
    idx = np.unique(np.concatenate([uni, cand, [0, n - 1]]))
    return idx.astype(np.int64)


def write(name, g, res, seed, extra):
    shape = (g.grid.s,) * g.grid.dim
    idx = sample_states(g.n, res.alpha, shape[::-1], seed)
    tied = oracle.tied_states(g, res.v, res.alpha)
    out = {
        "source": "oracle fixed point, written by tests/golden/make_fullsize.py",
        "n": int(g.n), "m1": int(g.m1), "m2": int(g.m2),
        "residual": float(res.residual), "outer": int(res.outer),
        "inner_total": int(res.inner_total), "converged": bool(res.converged),
        "oracle_seconds": float(res.seconds),
        "idx": idx.tolist(),
        "v": [float(x) for x in res.v[idx]],
        "alpha": [int(x) for x in res.alpha[idx]],
        "beta": [int(x) for x in res.beta[idx]],
        "tied": [bool(x) for x in tied[idx]],
        "vmax_abs": float(np.abs(res.v).max()),
        "tied_fraction": float(tied.mean()),
    }
    out.update(extra)
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {path}: {len(idx)} states, residual {res.residual:.3e}, "
          f"outer {res.outer}, inner {res.inner_total}, {res.seconds:.1f}s", flush=True)


def obstacle():
    levels = configs.c1_levels(points=1025, coarsest_points=33)
    t = time.perf_counter()
    results = oracle.famg_pi(levels, eps=0.0, c=1e-2)
    g = levels[-1]
    res = results[-1]
    contact = float(np.mean(res.alpha == 0))
    write("obstacle_1025.json", g, res, seed=1025, extra=
          {"workload": "obstacle 1025x1025 points, seed 1, lambda 0.5, FAMGpi c=1e-2",
           "points": [lv.meta["points"] for lv in levels],
           "per_level_outer": [r.outer for r in results],
           "contact_fraction": contact,
           "total_seconds": time.perf_counter() - t})


def write_full(name, g, res):
    """Every state of the oracle's fixed point: the value truncated to 36 of
    its 52 mantissa bits (relative error below 2^-36 = 1.5e-11, far below the
    parity bars), both strategies and the tie flags, in a compressed archive.
    The value's six high bytes are stored plane by plane (all most significant
    bytes first), which compresses the slowly varying high bytes of a smooth
    value."""
    v = np.ascontiguousarray(res.v, dtype=np.float64)
    bits = v.view(np.uint64) & ~np.uint64((1 << 16) - 1)     # the two low bytes are not stored
    planes = bits.view(np.uint8).reshape(-1, 8)[:, ::-1].T.copy()   # byte planes, most significant first
    tied = oracle.tied_states(g, res.v, res.alpha)
    path = os.path.join(HERE, name)
    np.savez_compressed(path, v_planes=planes[:6], n=np.int64(g.n), alpha=res.alpha.astype(np.uint8),
                        beta=res.beta.astype(np.uint8), tied=np.packbits(tied),
                        residual=np.float64(res.residual), vmax_abs=np.float64(np.abs(res.v).max()))
    print(f"wrote {path}: {os.path.getsize(path) / 1e6:.1f} MB", flush=True)


def isaacs3d():
    g = configs.c2(s=129)
    res = oracle.policy_iteration(g, eps=0.0, solver="krylov")
    write("isaacs3d_129.json", g, res, seed=129, extra=
          {"workload": "Isaacs 3-D 129^3 interior, seed 2, lambda 1, PI with Krylov evaluations"})
    write_full("isaacs3d_129_full.npz", g, res)


if __name__ == "__main__":
    what = sys.argv[1:] or ["obstacle", "isaacs3d"]
    for w in what:
        {"obstacle": obstacle, "isaacs3d": isaacs3d}[w]()
