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
# HBM-streaming kernel families reported on the finest level
STREAMING = ("smooth", "resid", "resid64", "improve")
CALIB_BYTES = 1 << 30  # bytes read (and written) by the calibration kernel


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


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=1025)
    ap.add_argument("--cpu-points", type=int, default=1025)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--amgpi", action="store_true")
    ap.add_argument("--roofline-kernel", default="auto")
    ap.add_argument("--forcing", type=float, default=0.1)
    ap.add_argument("--reuse", type=float, default=0.5)
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2", "c3", "c4"])
    ap.add_argument("--games", type=int, default=256, help="C3 batch size")
    ap.add_argument("--requests", type=int, default=100, help="C4 requests")
    ap.add_argument("--side", type=int, default=129, help="C2 interior points per side")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise kernel of known traffic (reads and writes "
                         f"{CALIB_BYTES >> 20} MiB): the reference for hardware byte counters")
    return ap.parse_args()


def main() -> int:
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding across GPUs is not implemented)"}))
        return 2
    return {"c0": run_c0, "c1": run_c1, "c2": run_c2, "c3": run_c3, "c4": run_c4}[args.workload](args)


def base_record(args, value, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_obstacle1025_famg_fp64.json")


def measured_traffic(family):
    """HBM bytes per launch of a kernel family from the committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    from paper_1107_1653_amd import rocprof_summary
    try:
        with open(TRAFFIC_FILE) as f:
            d = json.load(f)
    except OSError:
        return None, "no counter summary"
    if d.get("source_sha256") != rocprof_summary.source_hash():
        return None, "kernel sources changed since the counters were taken"
    fam = d.get("families", {}).get(family)
    if fam is None:
        return None, "family not in the counter summary"
    return fam["bytes_per_launch"], os.path.relpath(TRAFFIC_FILE, ROOT)


def calibration_kernel():
    """torch.neg over CALIB_BYTES of float32: one kernel that reads and writes
    exactly CALIB_BYTES each (counter runs scale by what it reads)."""
    import torch
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def run_c1(args) -> int:

    import torch  # device synchronisation around the timed region only
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    if args.calibrate_copy:
        calibration_kernel()

    t0 = time.perf_counter()
    levels = configs.c1_levels(points=args.points, coarsest_points=33)
    n = levels[-1].n
    log(f"[bench] generated {len(levels)} grids up to n={n} in {time.perf_counter() - t0:.1f}s")
    hs = [P.create_from(g) for g in levels]
    H = P.shapley_game_create_hierarchy(hs)
    a0 = np.zeros(levels[0].n, np.int32)

    def opts(prec):
        # inexact policy iteration: each linear solve to 0.1 x the previous
        # Shapley residual; AMG splitting reused while < 50% of policies change
        return P.shapley_default_opts(eps=1e-8, precision=prec, method=P.SHAPLEY_FAMGPI, alpha0=a0,
                                      beta0=a0, max_outer=5000, max_inner=5000, forcing=args.forcing,
                                      reuse_frac=args.reuse)

    o64 = opts(P.SHAPLEY_FP64)
    # pick the kernel family with the largest device time (one probed solve)
    fam = args.roofline_kernel
    if fam == "auto":
        for k in P.PROBE:
            P.shapley_probe_enable(k, True)
        log("[bench] probing kernel families (one solve)")
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
    for k in range(args.steps):
        t = time.perf_counter()
        st = P.shapley_solve(H, o64)
        lat.append(time.perf_counter() - t)
        log(f"[bench] step {k}: {1e3 * lat[-1]:.1f} ms")
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
    # the streaming kernels on the finest grid's level 0, timed with HIP
    # events in one more (untimed) solve: relaxation, cycle residual, FP64
    # residual, policy improvement
    for k in STREAMING:
        P.shapley_probe_enable(k, True)
    P.shapley_solve(H, o64)
    streaming = {}
    for k in STREAMING:
        r = P.shapley_probe_read_large(k, 0.5)
        P.shapley_probe_enable(k, False)
        if r["launches"] == 0:
            continue
        gbs = r["bytes"] / (r["ms"] * 1e-3) / 1e9
        streaming[k] = {"achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "launches": r["launches"],
                        "avg_launch_us": 1e3 * r["ms"] / r["launches"],
                        "alg_bytes_per_launch": r["bytes"] / r["launches"]}
    log("[bench] finest-level streaming kernels: " +
        ", ".join(f"{k} {v['achieved']:.0f} GB/s ({v['avg_launch_us']:.1f} us)" for k, v in streaming.items()))
    # sizes of the finest grid's first AMG levels (the launches above)
    first = P.shapley_hierarchy_level(H, 0, sizes_only=True)
    fine_levels = []
    for lvl in range(min(3, first["levels"])):
        d = P.shapley_hierarchy_level(H, lvl, sizes_only=True)
        fine_levels.append({"level": lvl, "n": int(d["n"]), "nnz": int(d["nnz"])})
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
    traffic, tsrc = measured_traffic(fam)
    roof = {"bound": "hbm", "kernel": fam, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": tsrc,
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
        "streaming": {"peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "launches": "launches moving at least half the largest algorithmic bytes of the family "
                                  f"(the first AMG levels of the {args.points}x{args.points} grid), HIP events",
                      "levels": fine_levels, "kernels": streaming},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    P.shapley_game_destroy(H)
    print(json.dumps(out), flush=True)
    return 0




def _opts(P, prec, args, **kw):
    return P.shapley_default_opts(eps=1e-8, precision=prec, max_outer=5000, max_inner=5000,
                                  forcing=args.forcing, reuse_frac=args.reuse, **kw)


def run_c0(args) -> int:
    """Isaacs 2-D, 33x33 interior grid (n = 1089): plain PI latency over
    at least 20 repeats, FP64 and mixed."""
    import torch
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    g = configs.c0()
    h = P.create_from(g)
    reps = max(args.steps, 20)
    out = {}
    for name, prec in (("fp64", P.SHAPLEY_FP64), ("mixed", P.SHAPLEY_MIXED)):
        o = _opts(P, prec, args)
        for _ in range(max(args.warmup, 1)):
            P.shapley_solve(h, o)
        torch.cuda.synchronize()
        lat = []
        for _ in range(reps):
            t = time.perf_counter()
            st = P.shapley_solve(h, o)
            lat.append(time.perf_counter() - t)
        lat = 1e3 * np.array(lat)
        out[name] = {"value": g.n / (np.mean(lat) * 1e-3), "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "residual": st["residual"],
                     "outer": st["outer"], "inner": st["inner_total"]}
    P.shapley_game_destroy(h)
    rec = base_record(args, out["fp64"]["value"], out["fp64"]["p50_ms"], "f64",
                      {"workload": "Isaacs 2-D 33x33 interior (n=1089), AMGpi FP64 to 1e-8", "repeats": reps})
    rec["latency_ms"] = {"p50": out["fp64"]["p50_ms"], "p99": out["fp64"]["p99_ms"]}
    rec["extra"] = out
    print(json.dumps(rec), flush=True)
    return 0


def run_c2(args) -> int:
    """Isaacs 3-D on 129^3: FP64 V-cycles vs FP32 V-cycles under FP64
    refinement, AMGpi to 1e-8; the mixed result's distance to the FP64 one."""
    import torch
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    t0 = time.perf_counter()
    g = configs.c2(s=args.side)
    log(f"[bench] generated C2 n={g.n} in {time.perf_counter() - t0:.1f}s")
    h = P.create_from(g)
    out, vals = {}, {}
    for name, prec in (("fp64", P.SHAPLEY_FP64), ("mixed", P.SHAPLEY_MIXED)):
        o = _opts(P, prec, args)
        for _ in range(args.warmup):
            P.shapley_solve(h, o)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t = time.perf_counter()
            st = P.shapley_solve(h, o)
            ts.append(time.perf_counter() - t)
        vals[name] = P.shapley_get_value(h)
        out[name] = {"value": g.n / float(np.mean(ts)), "ms_per_step": 1e3 * float(np.mean(ts)),
                     "residual": st["residual"], "outer": st["outer"], "inner": st["inner_total"],
                     "cycles": st["cycles_total"], "levels": st["levels"], "op_complexity": st["op_complexity"],
                     "setup_ms": 1e3 * st["setup_seconds"], "cycle_ms": 1e3 * st["cycle_seconds"]}
        log(f"[bench] C2 {name}: {out[name]['ms_per_step']:.1f} ms, residual {st['residual']:.1e}")
    out["mixed"]["max_abs_diff_vs_fp64"] = float(np.max(np.abs(vals["mixed"] - vals["fp64"])))
    P.shapley_game_destroy(h)
    rec = base_record(args, out["fp64"]["value"], out["fp64"]["ms_per_step"], "f64",
                      {"workload": f"Isaacs 3-D {args.side}^3 interior (n={g.n}), AMGpi to 1e-8"})
    rec["extra"] = out
    print(json.dumps(rec), flush=True)
    return 0


def run_c3(args) -> int:
    """256 independent 2-D Isaacs games (sides 65/129/257): one lock-step
    batched solve (one launch per kernel and level for all games) vs the same
    games solved one after another, FP64 and mixed."""
    import torch
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    t0 = time.perf_counter()
    side, lam = configs.c3_sizes(count=args.games)
    gs = [configs.c3_game(k, side[k], lam[k]) for k in range(args.games)]
    total = int(sum(g.n for g in gs))
    log(f"[bench] generated {len(gs)} games, sum n = {total} in {time.perf_counter() - t0:.1f}s")
    hs = [P.create_from(g) for g in gs]
    out = {}
    vals = {}
    for name, prec in (("batched_fp64", P.SHAPLEY_FP64), ("batched_mixed", P.SHAPLEY_MIXED)):
        o = _opts(P, prec, args)
        for _ in range(args.warmup):
            P.shapley_solve_batch(hs, o)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t = time.perf_counter()
            st = P.shapley_solve_batch(hs, o)
            ts.append(time.perf_counter() - t)
        vals[name] = [P.shapley_get_value(h) for h in hs[:8]]
        out[name] = {"value": total / float(np.mean(ts)), "ms_per_step": 1e3 * float(np.mean(ts)),
                     "max_residual": max(s["residual"] for s in st),
                     "max_outer": max(s["outer"] for s in st)}
        log(f"[bench] C3 {name}: {out[name]['ms_per_step']:.1f} ms")
    o = _opts(P, P.SHAPLEY_FP64, args)
    for h in hs[:4]:
        P.shapley_solve(h, o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for h in hs:
        P.shapley_solve(h, o)
    dt = time.perf_counter() - t
    seq = [P.shapley_get_value(h) for h in hs[:8]]
    out["sequential_fp64"] = {"value": total / dt, "ms_per_step": 1e3 * dt}
    log(f"[bench] C3 sequential fp64: {1e3 * dt:.1f} ms")
    out["batched_vs_alone_max_rel_diff"] = float(max(
        np.max(np.abs(a - b)) / np.max(np.abs(b)) for a, b in zip(vals["batched_fp64"], seq)))
    for h in hs:
        P.shapley_game_destroy(h)
    rec = base_record(args, out["batched_mixed"]["value"], out["batched_mixed"]["ms_per_step"], "f64",
                      {"workload": f"{len(gs)} Isaacs 2-D games, sides 65/129/257 (sum n={total}), "
                                   "batched AMGpi mixed to 1e-8", "games": len(gs)})
    rec["extra"] = out
    print(json.dumps(rec), flush=True)
    return 0


def run_c4(args) -> int:
    """Serving: Poisson arrivals of Isaacs (AMGpi) and obstacle (FAMGpi on a
    non-nested hierarchy) requests, sides log-uniform in [33, 1025], through
    the continuous-batching server with a 200 GB budget.  First a closed loop
    (everything queued at once) gives the saturation rate X_sat; then open
    loops at 0.5 and 0.8 X_sat report p50/p99 latency and solves/s."""
    import torch
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    reqs = configs.c4_requests(count=args.requests)
    t0 = time.perf_counter()
    handles, sizes = [], []
    for kind, side, lam, seed in reqs:
        if kind == 0:
            h = P.create_from(configs.c4_game(kind, side, lam, seed))
            handles.append((h, False, None))
        else:
            lv = configs.obstacle_levels_for_side(side, seed, lam)
            H = P.shapley_game_create_hierarchy([P.create_from(g) for g in lv])
            handles.append((H, True, lv[0].n))
        sizes.append(side * side)
    total = int(sum(sizes))
    log(f"[bench] created {len(handles)} requests (sum n = {total}) in {time.perf_counter() - t0:.1f}s")

    def opts_for(is_h, n0):
        if is_h:
            a0 = np.zeros(n0, np.int32)
            return _opts(P, P.SHAPLEY_MIXED, args, method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0)
        return _opts(P, P.SHAPLEY_MIXED, args)

    opts = [opts_for(is_h, n0) for (_, is_h, n0) in handles]

    def run(rate):
        srv = P.shapley_server_create(200 * 10 ** 9)
        rng = np.random.default_rng(7)
        arrivals = (np.zeros(len(handles)) if rate is None
                    else np.cumsum(rng.exponential(1.0 / rate, size=len(handles))))
        torch.cuda.synchronize()
        start = time.perf_counter()
        tickets = [None] * len(handles)
        sub_t = [0.0] * len(handles)
        nxt = 0
        done = 0
        lat = [None] * len(handles)
        while done < len(handles):
            now = time.perf_counter() - start
            while nxt < len(handles) and arrivals[nxt] <= now:
                tickets[nxt] = P.shapley_server_submit(srv, handles[nxt][0], opts[nxt])
                sub_t[nxt] = arrivals[nxt]
                nxt += 1
            active = P.shapley_server_step(srv)
            for i in range(nxt):
                if lat[i] is None:
                    st = P.shapley_server_poll(srv, tickets[i])
                    if st is not None:
                        lat[i] = (time.perf_counter() - start) - sub_t[i]
                        done += 1
            if active == 0 and nxt < len(handles):
                time.sleep(max(0.0, min(0.01, arrivals[nxt] - (time.perf_counter() - start))))
        wall = time.perf_counter() - start
        P.shapley_server_destroy(srv)
        lat = 1e3 * np.array(lat)
        return {"solves_per_s": len(handles) / wall, "unknowns_per_s": total / wall, "wall_s": wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}

    run(None)  # warm-up pass (allocations)
    closed = run(None)
    log(f"[bench] C4 closed loop: {closed}")
    xs = closed["solves_per_s"]
    o5 = run(0.5 * xs)
    log(f"[bench] C4 open loop 0.5 X_sat: {o5}")
    o8 = run(0.8 * xs)
    log(f"[bench] C4 open loop 0.8 X_sat: {o8}")
    for h, _, _ in handles:
        P.shapley_game_destroy(h)
    rec = base_record(args, closed["unknowns_per_s"], 1e3 * closed["wall_s"], "f64",
                      {"workload": f"{len(handles)} serving requests (50/50 Isaacs/obstacle, sides log-uniform "
                                   f"33..1025, sum n={total}), mixed precision, 200 GB budget",
                       "requests": len(handles)})
    rec["latency_ms"] = {"p50": o8["p50_ms"], "p99": o8["p99_ms"], "load": "0.8 X_sat"}
    rec["extra"] = {"closed_loop": closed, "open_0.5": o5, "open_0.8": o8}
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
