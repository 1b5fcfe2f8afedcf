#!/usr/bin/env python3
"""Throughput benchmark: unknowns solved per second to a 1e-8 Shapley residual.

Workload (one "step" = one complete solve): the obstacle problem
min(-0.5 Lap v + lambda v - f, v - psi) = 0 on 1025 x 1025 points
(1,046,529 unknowns, lambda = 0.5, f = 8 seeded Gaussian bumps,
psi = 0.2 sin(pi x1) sin(pi x2)), solved by full multilevel policy iteration
(FAMGpi, coarse grids 33, 65, ..., 1025 points, eps_l = 1e-2 h_l^2) to
||F(v) - v||_inf <= 1e-8 in FP64, with the data resident on the GPU.  The
same solve in mixed precision (FP32 V-cycles, FP64 refinement) is reported
beside it; `--amgpi` adds single-grid AMGpi from "stop everywhere".

Prints one JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns solved/s to 1e-8 Shapley residual, FP64 vs mixed; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(points: int) -> dict:
    """The oracle (plain FP64 CPU FAMGpi with SuperLU) on a smaller grid of the
    same obstacle workload, one thread, in a child process."""
    code = f"""
import json, sys, time
sys.path.insert(0, {ROOT!r})
import numpy as np
from shapley_inputs import configs
import oracle
levels = configs.c1_levels(points={points}, coarsest_points=33)
a0 = np.zeros(levels[0].n, np.int32)
t = time.perf_counter()
res = oracle.famg_pi(levels, eps=1e-8, c=1e-2, alpha0=a0, beta0=a0)
dt = time.perf_counter() - t
print(json.dumps(dict(seconds=dt, n=levels[-1].n, residual=res[-1].residual)))
"""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    if out.returncode != 0:
        raise RuntimeError(out.stderr)
    d = json.loads(out.stdout.strip().splitlines()[-1])
    return {
        "value": d["n"] / d["seconds"],
        "unit": "unknowns/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"obstacle workload at {points}x{points} points (n={d['n']}), oracle FAMGpi "
                   f"(SuperLU per policy) to 1e-8, {d['seconds']:.2f} s, residual {d['residual']:.1e}"),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=1025)
    ap.add_argument("--cpu-points", type=int, default=513)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--amgpi", action="store_true")
    ap.add_argument("--roofline-kernel", default="auto")
    ap.add_argument("--forcing", type=float, default=0.1)
    ap.add_argument("--reuse", type=float, default=0.05)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2

    import torch  # device synchronisation around the timed region only
    import paper_1107_1653_amd as P
    from shapley_inputs import configs

    t0 = time.perf_counter()
    levels = configs.c1_levels(points=args.points, coarsest_points=33)
    n = levels[-1].n
    log(f"[bench] generated {len(levels)} grids up to n={n} in {time.perf_counter() - t0:.1f}s")
    hs = [P.create_from(g) for g in levels]
    H = P.shapley_game_create_hierarchy(hs)
    a0 = np.zeros(levels[0].n, np.int32)

    def opts(prec):
        # inexact policy iteration: each linear solve to 0.1 x the previous
        # Shapley residual; AMG splitting reused while < 5% of policies change
        return P.shapley_default_opts(eps=1e-8, precision=prec, method=P.SHAPLEY_FAMGPI, alpha0=a0,
                                      beta0=a0, max_outer=5000, max_inner=5000, forcing=args.forcing,
                                      reuse_frac=args.reuse)

    o64 = opts(P.SHAPLEY_FP64)
    # pick the kernel family with the largest device time (one probed solve)
    fam = args.roofline_kernel
    if fam == "auto":
        for k in P.PROBE:
            P.shapley_probe_enable(k, True)
        P.shapley_solve(H, o64)
        tot = {k: P.shapley_probe_read(k)["ms"] for k in P.PROBE}
        for k in P.PROBE:
            P.shapley_probe_enable(k, False)
        fam = max(tot, key=tot.get)
        log(f"[bench] per-family device ms of one solve: " +
            ", ".join(f"{k}={v:.1f}" for k, v in sorted(tot.items(), key=lambda kv: -kv[1])))

    for _ in range(args.warmup):
        P.shapley_solve(H, o64)
    P.shapley_probe_enable(fam, True)
    torch.cuda.synchronize()
    lat = []
    st = None
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        st = P.shapley_solve(H, o64)
        lat.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    pr = P.shapley_probe_read(fam)
    P.shapley_probe_enable(fam, False)
    ms_per_step = 1e3 * wall / args.steps
    value = n / (wall / args.steps)
    log(f"[bench] FAMGpi FP64: {ms_per_step:.1f} ms/solve, residual {st['residual']:.2e}, "
        f"outer {st['outer']}, cycles {st['cycles_total']}")

    extra = {}
    if not args.no_mixed:
        om = opts(P.SHAPLEY_MIXED)
        P.shapley_solve(H, om)
        lm = []
        for _ in range(args.steps):
            t = time.perf_counter()
            sm = P.shapley_solve(H, om)
            lm.append(time.perf_counter() - t)
        vm = P.shapley_get_value(H)
        extra["mixed"] = {"value": n / float(np.mean(lm)), "ms_per_step": 1e3 * float(np.mean(lm)),
                          "residual": sm["residual"]}
        log(f"[bench] FAMGpi mixed: {1e3 * np.mean(lm):.1f} ms/solve, residual {sm['residual']:.2e}")
    v64 = None
    P.shapley_solve(H, o64)
    v64 = P.shapley_get_value(H)
    if not args.no_mixed:
        extra["mixed"]["max_abs_diff_vs_fp64"] = float(np.max(np.abs(vm - v64)))
    if args.amgpi:
        g = levels[-1]
        h = P.create_from(g)
        oa = P.shapley_default_opts(eps=1e-8, alpha0=np.zeros(n, np.int32), beta0=np.zeros(n, np.int32),
                                    max_outer=5000, forcing=args.forcing, reuse_frac=args.reuse)
        t = time.perf_counter()
        sa = P.shapley_solve(h, oa)
        dt = time.perf_counter() - t
        extra["amgpi_fp64"] = {"value": n / dt, "seconds": dt, "outer": sa["outer"]}
        P.shapley_game_destroy(h)
        log(f"[bench] AMGpi FP64: {dt:.2f} s, outer {sa['outer']}")

    achieved = (pr["bytes"] / max(pr["launches"], 1)) / (pr["ms"] / max(pr["launches"], 1) * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": fam, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "launches": pr["launches"], "avg_launch_us": 1e3 * pr["ms"] / max(pr["launches"], 1),
            "alg_bytes_per_launch": pr["bytes"] / max(pr["launches"], 1)}

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.cpu_points)
        except Exception as e:  # the GPU number stands on its own
            log(f"[bench] cpu baseline failed: {e}")
    lat_ms = 1e3 * np.array(lat)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"obstacle VI {args.points}x{args.points} points (n={n}), FAMGpi FP64 to 1e-8",
                   "n": n, "eps": 1e-8, "grids": [g.meta["points"] for g in levels],
                   "forcing": args.forcing, "reuse_frac": args.reuse},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "solve": {"outer": st["outer"], "inner": st["inner_total"], "cycles": st["cycles_total"],
                  "residual": st["residual"], "setup_ms": 1e3 * st["setup_seconds"],
                  "cycle_ms": 1e3 * st["cycle_seconds"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    P.shapley_game_destroy(H)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
