"""Writes the full-size parity fixture of the 3-D Isaacs game from the
oracle alone.

    python tests/golden/make_fullsize.py   # -> isaacs3d_129_full.npz

isaacs3d_129_full.npz holds the oracle's fixed point at every state of the
3-D Isaacs game with 129 interior points per side (value, strategies of both
players, tie flags): oracle policy iteration (Sec. 4.2) from the default
start with the Krylov policy evaluation (the sparse LU does not fit in memory
at this size), eps = 0.  The oracle takes minutes here, too long to run
beside a GPU test; the other full-size workloads are solved by the oracle in
worker processes while the GPU test runs.

Only the seeded generators and `oracle` are used.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from shapley_inputs import configs  # noqa: E402


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
    print(f"oracle: residual {res.residual:.3e}, outer {res.outer}, inner {res.inner_total}, {res.seconds:.1f}s",
          flush=True)
    write_full("isaacs3d_129_full.npz", g, res)


if __name__ == "__main__":
    isaacs3d()
