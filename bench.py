#!/usr/bin/env python3
"""Throughput benchmark: unknowns solved per second to a 1e-8 Shapley residual.

Default workload (one "step" = one complete batched solve): 256 independent
2-D Isaacs games, grid sides drawn from {65, 129, 257} interior points
(sum n = 7,540,224 unknowns), lambda log-uniform in [0.1, 10], seeded
f = sin(2 pi x1) cos(2 pi x2) + 0.1 N(0,1), solved together by batched
policy iteration with the algebraic-multigrid inner solve (one launch per
kernel and level for all games), FP32 V-cycles under FP64 refinement, to
||F(v) - v||_inf <= 1e-8 per game, with the data resident on the GPU.  The
same batch in FP64, and the games solved one by one in FP64 (plain GPU
policy iteration), are reported beside it.  The 3-D Isaacs game on 129^3
(FP64 and mixed) and the obstacle problem on 1025 x 1025 points (FAMGpi) are
reported in `extra`, each with its own roofline.  `--workload` picks one of
c0 (Isaacs 33^2 latency), c1 (obstacle), c2 (3-D Isaacs), c3 (the default),
c4 (serving stream), two_stopper (the paper's 1-D example, AMGpi vs FAMGpi),
general (a point-cloud game without a grid) or iex1 (the paper's Isaacs
example with continuous action sets) as the headline instead.

Prints one JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns solved/s to 1e-8 Shapley residual, FP64 vs mixed; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
CALIB_BYTES = 1 << 30  # bytes read (and written) by the calibration kernel
# the limiter of each kernel family: streaming kernels are bound by HBM
# bandwidth; the Galerkin product, interpolation and the one-workgroup V-cycle
# tail are irregular, latency-bound kernels (reported against the HBM peak)
BOUND = {"smooth": "hbm", "resid": "hbm", "resid64": "hbm", "improve": "hbm", "restrict": "hbm",
         "prolong": "hbm", "rap": "latency", "interp": "latency", "tail": "latency"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3",
                    choices=["c0", "c1", "c2", "c3", "c4", "two_stopper", "general", "iex1"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline's timed steps only (for kernel traces): no FP64 or one-by-one runs")
    ap.add_argument("--forcing", type=float, default=0.2)
    ap.add_argument("--reuse", type=float, default=0.5)
    ap.add_argument("--nu1", type=int, default=1, help="relaxation sweeps before the coarse correction")
    ap.add_argument("--nu2", type=int, default=2, help="relaxation sweeps after the coarse correction")
    ap.add_argument("--games", type=int, default=256, help="C3 batch size")
    ap.add_argument("--requests", type=int, default=1000, help="C4 requests")
    ap.add_argument("--side", type=int, default=129, help="C2 interior points per side")
    ap.add_argument("--points", type=int, default=1025, help="C1 points per side")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise kernel of known traffic (reads and writes "
                         f"{CALIB_BYTES >> 20} MiB): the reference for hardware byte counters")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# measurement helpers
# ---------------------------------------------------------------------------

def sync():
    import torch
    torch.cuda.synchronize()


def calibration_kernel():
    """torch.neg over CALIB_BYTES of float32: one kernel that reads and writes
    exactly CALIB_BYTES each (counter runs scale by what it reads)."""
    import torch
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    sync()
    torch.neg(x, out=y)
    sync()
    del x, y


def family_profile(P, solve):
    """One (untimed) solve with every kernel family probed by HIP events:
    per family the device time of all launches and of its largest launches
    (at least half the largest algorithmic bytes: the finest AMG level)."""
    for k in P.PROBE:
        P.shapley_probe_enable(k, True)
    solve()
    out = {}
    for k in P.PROBE:
        a = P.shapley_probe_read(k)
        b = P.shapley_probe_read_large(k, 0.5)
        P.shapley_probe_enable(k, False)
        if a["launches"] == 0:
            continue
        out[k] = {"total_ms": a["ms"], "launches": a["launches"], "large_launches": b["launches"],
                  "large_avg_us": 1e3 * b["ms"] / max(b["launches"], 1),
                  "large_alg_bytes_per_launch": b["bytes"] / max(b["launches"], 1),
                  "large_gbs": b["bytes"] / max(b["ms"] * 1e-3, 1e-30) / 1e9}
        out[k]["large_frac"] = out[k]["large_gbs"] / HBM_PEAK_GBS
    return out


def timed(P, solve, steps, warmup, probe_family=None):
    """`warmup` untimed solves, then `steps` timed ones between device
    synchronisations; with probe_family, that family's launches are bracketed
    by HIP events on their stream during the timed solves."""
    for _ in range(warmup):
        solve()
    sync()
    if probe_family:
        P.shapley_probe_enable(probe_family, True)
    lat = []
    st = None
    t0 = time.perf_counter()
    for k in range(steps):
        t = time.perf_counter()
        st = solve()
        lat.append(time.perf_counter() - t)
    sync()
    wall = time.perf_counter() - t0
    pr = None
    if probe_family:
        pr = P.shapley_probe_read_large(probe_family, 0.5)
        P.shapley_probe_enable(probe_family, False)
    return wall, np.array(lat), st, pr


def traffic_for(workload, family):
    """HBM bytes per launch (largest launches of the family) from the
    committed counter summary of this workload, or None when it is missing or
    the kernel sources changed since the counters were taken."""
    from paper_1107_1653_amd import rocprof_summary
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None, "no counter summary"
    if d.get("source_sha256") != rocprof_summary.source_hash():
        return None, "kernel sources changed since the counters were taken"
    fam = d.get("families", {}).get(family)
    if fam is None:
        return None, "family not in the counter summary"
    return fam["bytes_per_launch"], os.path.relpath(path, ROOT)


def roofline(workload, fam, pr):
    """The roofline object of a kernel family from its probed launches."""
    n = max(pr["launches"], 1)
    bpl = pr["bytes"] / n
    avg_s = pr["ms"] * 1e-3 / n
    achieved = bpl / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic, src = traffic_for(workload, fam)
    return {"bound": BOUND.get(fam, "hbm"), "kernel": fam, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": src,
            "launches": pr["launches"], "avg_launch_us": 1e6 * avg_s, "alg_bytes_per_launch": bpl,
            "launch_set": "the family's launches moving at least half its largest algorithmic bytes "
                          "(finest AMG level), HIP events on the launch stream over the timed steps"}


def dominant(fams):
    return max(fams, key=lambda k: fams[k]["total_ms"])


def mu_max(g):
    csum = np.concatenate([[0.0], np.cumsum(g.w)])
    rows = csum[g.row_ptr[1:]] - csum[g.row_ptr[:-1]]
    return g.mu * float(rows.max())


def record(args, value, ms_per_step, dtype, config, steps=None):
    return {"metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1,
            "steps": args.steps if steps is None else steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def opts(P, args, prec, **kw):
    # inexact policy iteration: each linear solve to `forcing` x the previous
    # Shapley residual; AMG splitting reused while < 50% of the policies
    # changed; V(nu1, nu2) cycles
    return P.shapley_default_opts(eps=1e-8, precision=prec, max_outer=5000, max_inner=5000, forcing=args.forcing,
                                  reuse_frac=args.reuse, nu1=args.nu1, nu2=args.nu2, **kw)


def measure(P, args, workload, solve, steps=None):
    """Family profile, then the timed steps with the dominant family probed;
    returns (wall, latencies, stats, roofline, families)."""
    fams = family_profile(P, solve)
    fam = dominant(fams)
    log(f"[bench] {workload}: per-family device ms of one solve: " +
        ", ".join(f"{k}={v['total_ms']:.1f}" for k, v in sorted(fams.items(), key=lambda kv: -kv[1]['total_ms'])))
    wall, lat, st, pr = timed(P, solve, args.steps if steps is None else steps, args.warmup, fam)
    return wall, lat, st, roofline(workload, fam, pr), fams


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def c3_line(args):
    """256 2-D Isaacs games, batched mixed (headline), batched FP64 and one
    by one in FP64."""
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    t0 = time.perf_counter()
    side, lam = configs.c3_sizes(count=args.games)
    gs = [configs.c3_game(k, side[k], lam[k]) for k in range(args.games)]
    total = int(sum(g.n for g in gs))
    log(f"[bench] C3: generated {len(gs)} games, sum n = {total} in {time.perf_counter() - t0:.1f}s")
    sync()
    t = time.perf_counter()
    hs = [P.create_from(g) for g in gs]
    sync()
    create_s = time.perf_counter() - t
    om, o64 = opts(P, args, P.SHAPLEY_MIXED), opts(P, args, P.SHAPLEY_FP64)
    mixed = lambda: P.shapley_solve_batch(hs, om)
    wall, lat, st, roof, fams = measure(P, args, "c3", mixed)
    ms = 1e3 * wall / args.steps
    value = total / (wall / args.steps)
    log(f"[bench] C3 batched mixed: {ms:.1f} ms/batch, worst residual {max(s['residual'] for s in st):.1e}")
    v_mixed = [P.shapley_get_value(h) for h in hs]
    if args.headline_only:
        line = record(args, value, ms, "f32+f64", {"workload": "headline steps only", "sum_n": total})
        line["roofline"] = roof
        line["families"] = fams
        return line, gs, v_mixed
    # the same steps without any probe
    w2, _, _, _ = timed(P, mixed, args.steps, 0)
    w64, lat64, st64, _ = timed(P, lambda: P.shapley_solve_batch(hs, o64), args.steps, args.warmup)
    v64 = [P.shapley_get_value(h) for h in hs]
    log(f"[bench] C3 batched fp64: {1e3 * w64 / args.steps:.1f} ms/batch")
    # plain FP64 GPU policy iteration, one game after another
    for h in hs[:4]:
        P.shapley_solve(h, o64)
    sync()
    t = time.perf_counter()
    for h in hs:
        P.shapley_solve(h, o64)
    sync()
    seq = time.perf_counter() - t
    v_seq = [P.shapley_get_value(h) for h in hs]
    log(f"[bench] C3 one by one fp64: {1e3 * seq:.1f} ms")
    t = time.perf_counter()
    P.shapley_solve_batch(hs, om)
    vals = [P.shapley_get_value(h) for h in hs]
    e2e = time.perf_counter() - t + create_s
    for h in hs:
        P.shapley_game_destroy(h)
    line = record(args, value, ms, "f32+f64",
                  {"workload": f"{len(gs)} Isaacs 2-D games, interior sides 65/129/257 (sum n={total}), "
                               "batched AMGpi, FP32 V-cycles + FP64 refinement, to 1e-8",
                   "games": len(gs), "sum_n": total, "eps": 1e-8, "forcing": args.forcing,
                   "reuse_frac": args.reuse, "cycle": f"V({args.nu1},{args.nu2}) weighted Jacobi, omega 0.8"})
    line["latency_ms"] = {"p50": float(np.percentile(1e3 * lat, 50)), "p99": float(np.percentile(1e3 * lat, 99))}
    line["roofline"] = roof
    line["families"] = fams
    line["extra_c3"] = {
        "unprobed_ms_per_step": 1e3 * w2 / args.steps,
        "batched_fp64": {"value": total / (w64 / args.steps), "ms_per_step": 1e3 * w64 / args.steps,
                         "max_residual": max(s["residual"] for s in st64)},
        "one_by_one_fp64": {"value": total / seq, "ms": 1e3 * seq,
                            "what": "plain FP64 GPU policy iteration, the 256 games solved one after another"},
        "batched_mixed_vs_fp64_max_abs": float(max(np.max(np.abs(a - b)) for a, b in zip(v_mixed, v64))),
        "batched_vs_one_by_one_max_rel": float(max(np.max(np.abs(a - b)) / np.max(np.abs(b))
                                                   for a, b in zip(v64, v_seq))),
        "end_to_end_s": e2e, "create_s": create_s,
        "end_to_end_what": "create from host arrays + one batched mixed solve + values copied to the host",
        "max_residual": max(s["residual"] for s in st),
    }
    return line, gs, v_mixed


def c3_cpu_baseline(args, gs, v_gpu):
    """The oracle (FP64 policy iteration, SuperLU per policy) on every game of
    the batch, in worker processes over the host's cores, to the same 1e-8
    residual (about 10-15 s of wall time with 16 workers); also the error of
    the GPU's batched mixed values against it, game by game."""
    from oracle.jobs import Jobs
    from shapley_inputs import configs
    side, lam = configs.c3_sizes(count=args.games)
    pick = list(range(args.games))
    jobs = Jobs([(f"g{k}", "c3", [k, int(side[k]), float(lam[k])], 1e-8) for k in pick],
                cost=lambda j: float(j[2][1]) ** 3)
    res = jobs.wait(timeout=900, log=log)
    n = sum(gs[k].n for k in pick)
    err = max(float(np.max(np.abs(v_gpu[k] - res[f"g{k}"]["v"])) / np.max(np.abs(res[f"g{k}"]["v"]))) for k in pick)
    bound = max(1e-8 / (1.0 - mu_max(gs[k])) / np.max(np.abs(res[f"g{k}"]["v"])) for k in pick)
    cpu = {"value": n / jobs.seconds, "unit": "unknowns/s", "cores": jobs.workers, "kind": "oracle",
           "sample": f"all {len(pick)} games of the batch (sum n={n}), oracle policy iteration with "
                     f"SuperLU to 1e-8, {jobs.workers} worker processes, {jobs.seconds:.1f} s wall"}
    return cpu, {"games_compared": len(pick), "max_rel_err_vs_oracle": err,
                 "contraction_bound_rel": bound,
                 "what": "GPU batched mixed values vs the oracle, both stopped at ||F(v) - v|| <= 1e-8"}


def c2_line(args):
    """3-D Isaacs on 129^3: FP64 and mixed AMGpi; error against the oracle's
    stored fixed point at every state."""
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    t0 = time.perf_counter()
    g = configs.c2(s=args.side)
    log(f"[bench] C2: generated n={g.n} in {time.perf_counter() - t0:.1f}s")
    sync()
    t = time.perf_counter()
    h = P.create_from(g)
    sync()
    create_s = time.perf_counter() - t
    out, vals = {}, {}
    for name, prec in (("mixed", P.SHAPLEY_MIXED), ("fp64", P.SHAPLEY_FP64)):
        o = opts(P, args, prec)
        solve = lambda: P.shapley_solve(h, o)
        if name == "mixed":
            wall, lat, st, roof, fams = measure(P, args, "c2", solve)
        else:
            wall, lat, st, _ = timed(P, solve, args.steps, args.warmup)
        vals[name] = P.shapley_get_value(h)
        out[name] = {"value": g.n / (wall / args.steps), "ms_per_step": 1e3 * wall / args.steps,
                     "residual": st["residual"], "outer": st["outer"], "inner": st["inner_total"],
                     "cycles": st["cycles_total"], "levels": st["levels"], "op_complexity": st["op_complexity"]}
        log(f"[bench] C2 {name}: {out[name]['ms_per_step']:.1f} ms, residual {st['residual']:.1e}")
    P.shapley_game_destroy(h)
    err = None
    path = os.path.join(ROOT, "tests", "golden", "isaacs3d_129_full.npz")
    if args.side == 129 and os.path.exists(path):
        with np.load(path) as d:
            planes = d["v_planes"]
            b = np.zeros((g.n, 8), np.uint8)
            for k in range(planes.shape[0]):
                b[:, 7 - k] = planes[k]
            ref = b.view(np.float64).reshape(-1)
        err = {k: float(np.max(np.abs(v - ref)) / np.max(np.abs(ref))) for k, v in vals.items()}
        err["contraction_bound_rel"] = 1e-8 / (1.0 - mu_max(g)) / float(np.max(np.abs(ref)))
        err["what"] = "max over all states of |v - v*| / max |v*|, v* the oracle's stored fixed point"
    line = record(args, out["mixed"]["value"], out["mixed"]["ms_per_step"], "f32+f64",
                  {"workload": f"Isaacs 3-D {args.side}^3 interior (n={g.n}), AMGpi to 1e-8, FP32 V-cycles + FP64 "
                               "refinement", "n": g.n})
    line["roofline"] = roof
    line["families"] = fams
    line["fp64"] = out["fp64"]
    line["mixed"] = out["mixed"]
    line["mixed_vs_fp64_max_abs"] = float(np.max(np.abs(vals["mixed"] - vals["fp64"])))
    line["error_vs_oracle"] = err
    line["create_s"] = create_s
    return line


def c1_line(args, with_oracle=True):
    """Obstacle problem on 1025 x 1025 points, FAMGpi FP64 (and mixed);
    error against the oracle's FAMGpi fixed point at every state."""
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    levels = configs.c1_levels(points=args.points, coarsest_points=33)
    g = levels[-1]
    jobs = None
    if with_oracle:
        from oracle.jobs import Jobs
        jobs = Jobs([("c1", "c1", [args.points, 33], 0.0)])
    sync()
    t = time.perf_counter()
    H = P.shapley_game_create_hierarchy([P.create_from(x) for x in levels])
    sync()
    create_s = time.perf_counter() - t
    a0 = np.zeros(levels[0].n, np.int32)
    out, vals = {}, {}
    for name, prec in (("fp64", P.SHAPLEY_FP64), ("mixed", P.SHAPLEY_MIXED)):
        o = opts(P, args, prec, method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0)
        solve = lambda: P.shapley_solve(H, o)
        if name == "fp64":
            wall, lat, st, roof, fams = measure(P, args, "c1", solve)
        else:
            wall, lat, st, _ = timed(P, solve, args.steps, args.warmup)
        vals[name] = P.shapley_get_value(H)
        out[name] = {"value": g.n / (wall / args.steps), "ms_per_step": 1e3 * wall / args.steps,
                     "p50_ms": float(np.percentile(1e3 * lat, 50)), "p99_ms": float(np.percentile(1e3 * lat, 99)),
                     "residual": st["residual"], "outer": st["outer"], "cycles": st["cycles_total"]}
        log(f"[bench] C1 {name}: {out[name]['ms_per_step']:.1f} ms, residual {st['residual']:.1e}")
    P.shapley_game_destroy(H)
    line = record(args, out["fp64"]["value"], out["fp64"]["ms_per_step"], "f64",
                  {"workload": f"obstacle VI {args.points}x{args.points} points (n={g.n}), FAMGpi to 1e-8",
                   "grids": [x.meta["points"] for x in levels]})
    line["roofline"] = roof
    line["families"] = fams
    line["fp64"] = out["fp64"]
    line["mixed"] = out["mixed"]
    line["create_s"] = create_s
    if jobs is not None:
        ref = jobs.wait(timeout=600, log=log)["c1"]["v"]
        line["error_vs_oracle"] = {
            k: float(np.max(np.abs(v - ref)) / np.max(np.abs(ref))) for k, v in vals.items()}
        line["error_vs_oracle"]["contraction_bound_rel"] = 1e-8 / (1.0 - mu_max(g)) / float(np.max(np.abs(ref)))
        line["error_vs_oracle"]["what"] = "max over all states, oracle FAMGpi fixed point"
    return line


def c0_line(args):
    """Isaacs 2-D, 33x33 interior grid (n = 1089): plain PI latency over at
    least 20 repeats, FP64 and mixed."""
    import paper_1107_1653_amd as P
    import oracle
    from shapley_inputs import configs
    g = configs.c0()
    h = P.create_from(g)
    reps = max(args.steps, 20)
    out = {}
    for name, prec in (("fp64", P.SHAPLEY_FP64), ("mixed", P.SHAPLEY_MIXED)):
        o = opts(P, args, prec)
        wall, lat, st, _ = timed(P, lambda: P.shapley_solve(h, o), reps, max(args.warmup, 1))
        lat = 1e3 * lat
        out[name] = {"value": g.n / (np.mean(lat) * 1e-3), "p50_ms": float(np.percentile(lat, 50)),
                     "p99_ms": float(np.percentile(lat, 99)), "residual": st["residual"], "outer": st["outer"]}
    v = P.shapley_get_value(h)
    P.shapley_game_destroy(h)
    ref = oracle.policy_iteration(g, eps=1e-8)
    line = record(args, out["fp64"]["value"], out["fp64"]["p50_ms"], "f64",
                  {"workload": "Isaacs 2-D 33x33 interior (n=1089), AMGpi FP64 to 1e-8", "repeats": reps}, reps)
    line["latency_ms"] = {"p50": out["fp64"]["p50_ms"], "p99": out["fp64"]["p99_ms"]}
    line["extra"] = out
    line["error_vs_oracle"] = float(np.max(np.abs(v - ref.v)) / np.max(np.abs(ref.v)))
    return line


def c4_line(args):
    """Serving: Poisson arrivals of Isaacs (AMGpi) and obstacle (FAMGpi)
    requests, sides log-uniform in [33, 1025], through the request loop with a
    200 GB budget.  A closed loop (everything queued at once) gives the
    saturation rate X_sat; open loops at 0.5 and 0.8 X_sat give p50/p99
    latency; the same requests solved one after another by plain FP64 GPU
    policy iteration are the reference."""
    import paper_1107_1653_amd as P
    from shapley_inputs import configs
    reqs = configs.c4_requests(count=args.requests)
    t0 = time.perf_counter()
    handles, sizes = [], []
    for kind, side, lam, seed in reqs:
        if kind == 0:
            handles.append((P.create_from(configs.c4_game(kind, side, lam, seed)), False, None))
        else:
            lv = configs.obstacle_levels_for_side(side, seed, lam)
            handles.append((P.shapley_game_create_hierarchy([P.create_from(g) for g in lv]), True, lv[0].n))
        sizes.append(side * side)
    total = int(sum(sizes))
    log(f"[bench] C4: created {len(handles)} requests (sum n = {total}) in {time.perf_counter() - t0:.1f}s")

    def opts_for(is_h, n0, prec):
        if is_h:
            a0 = np.zeros(n0, np.int32)
            return opts(P, args, prec, method=P.SHAPLEY_FAMGPI, alpha0=a0, beta0=a0)
        return opts(P, args, prec)

    om = [opts_for(is_h, n0, P.SHAPLEY_MIXED) for (_, is_h, n0) in handles]

    def run(rate):
        srv = P.shapley_server_create(200 * 10 ** 9)
        rng = np.random.default_rng(7)
        arrivals = (np.zeros(len(handles)) if rate is None
                    else np.cumsum(rng.exponential(1.0 / rate, size=len(handles))))
        sync()
        start = time.perf_counter()
        tickets = [None] * len(handles)
        nxt = done = 0
        lat = [None] * len(handles)
        max_cohorts = 0
        while done < len(handles):
            now = time.perf_counter() - start
            while nxt < len(handles) and arrivals[nxt] <= now:
                tickets[nxt] = P.shapley_server_submit(srv, handles[nxt][0], om[nxt])
                nxt += 1
            active = P.shapley_server_step(srv)
            max_cohorts = max(max_cohorts, P.shapley_server_info(srv)["cohorts"])
            for i in range(nxt):
                if lat[i] is None:
                    st = P.shapley_server_poll(srv, tickets[i])
                    if st is not None:
                        lat[i] = (time.perf_counter() - start) - arrivals[i]
                        done += 1
            if active == 0 and nxt < len(handles):
                time.sleep(max(0.0, min(0.01, arrivals[nxt] - (time.perf_counter() - start))))
        wall = time.perf_counter() - start
        P.shapley_server_destroy(srv)
        lat = 1e3 * np.array(lat)
        return {"solves_per_s": len(handles) / wall, "unknowns_per_s": total / wall, "wall_s": wall,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "max_cohorts": max_cohorts}

    run(None)  # warm-up pass (engines and their workspaces)
    closed = run(None)
    log(f"[bench] C4 closed loop: {closed}")
    xs = closed["solves_per_s"]
    o5 = run(0.5 * xs)
    log(f"[bench] C4 open loop 0.5 X_sat: {o5}")
    o8 = run(0.8 * xs)
    log(f"[bench] C4 open loop 0.8 X_sat: {o8}")
    # plain FP64 GPU policy iteration, one request after another
    sync()
    t = time.perf_counter()
    for (h, is_h, n0) in handles:
        P.shapley_solve(h, opts_for(is_h, n0, P.SHAPLEY_FP64))
    sync()
    seq = time.perf_counter() - t
    log(f"[bench] C4 one by one fp64: {seq:.2f} s")
    for h, _, _ in handles:
        P.shapley_game_destroy(h)
    line = record(args, closed["unknowns_per_s"], 1e3 * closed["wall_s"], "f32+f64",
                  {"workload": f"{len(handles)} serving requests (50/50 Isaacs/obstacle, sides log-uniform "
                               f"33..1025, sum n={total}), mixed precision, 200 GB budget",
                   "requests": len(handles)}, 1)
    line["latency_ms"] = {"p50": o8["p50_ms"], "p99": o8["p99_ms"], "load": "0.8 X_sat"}
    line["extra"] = {"closed_loop": closed, "open_0.5": o5, "open_0.8": o8,
                     "one_by_one_fp64": {"unknowns_per_s": total / seq, "wall_s": seq,
                                         "what": "plain FP64 GPU policy iteration, requests one after another"}}
    return line


def two_stopper_line(args):
    """The paper's 1-D two-stopper game (Sec. 6.3) on 2049 points: AMGpi from
    'stop everywhere' vs FAMGpi on the grids 33 ... 2049, to 1e-10 as in the
    paper's tables; error against the closed form."""
    import paper_1107_1653_amd as P
    from shapley_inputs import games
    pts = [33, 65, 129, 257, 513, 1025, 2049]
    levels = [games.two_stopper_game(p) for p in pts]
    g = levels[-1]
    x = np.arange(1, pts[-1] - 1) / (pts[-1] - 1)
    u = games.two_stopper_exact(x)
    out = {}
    h = P.create_from(g)
    a0 = np.zeros(g.n, np.int32)
    oa = P.shapley_default_opts(eps=1e-10, alpha0=a0, beta0=a0, max_outer=5000, max_inner=5000)
    wall, lat, st, _ = timed(P, lambda: P.shapley_solve(h, oa), max(1, args.steps // 2), 0)
    out["amgpi"] = {"seconds": wall / max(1, args.steps // 2), "outer": st["outer"], "residual": st["residual"],
                    "err_inf": float(np.max(np.abs(P.shapley_get_value(h) - u)))}
    P.shapley_game_destroy(h)
    H = P.shapley_game_create_hierarchy([P.create_from(x_) for x_ in levels])
    c0 = np.zeros(levels[0].n, np.int32)
    of = P.shapley_default_opts(eps=1e-10, method=P.SHAPLEY_FAMGPI, alpha0=c0, beta0=c0, max_outer=5000,
                                max_inner=5000)
    wall, lat, st, _ = timed(P, lambda: P.shapley_solve(H, of), args.steps, args.warmup)
    out["famgpi"] = {"seconds": wall / args.steps, "outer": st["outer"], "residual": st["residual"],
                     "err_inf": float(np.max(np.abs(P.shapley_get_value(H) - u)))}
    P.shapley_game_destroy(H)
    log(f"[bench] two-stopper: {out}")
    line = record(args, g.n / out["famgpi"]["seconds"], 1e3 * out["famgpi"]["seconds"], "f64",
                  {"workload": "1-D two-stopper game, 2049 points (n=2047), FAMGpi on 33..2049 points to 1e-10",
                   "n": g.n})
    line["extra"] = out
    line["extra"]["famgpi_speedup_over_amgpi"] = out["amgpi"]["seconds"] / out["famgpi"]["seconds"]
    line["extra"]["paper"] = {"amgpi_outer": 841, "amgpi_s": 1740.0, "famgpi_s": 0.95, "err_inf": 1.16e-7,
                              "hardware": "serial C on an unstated CPU (context only)"}
    return line


def general_line(args):
    """A game without a grid: 2^18 random points of the unit square, each
    moving to its 8 nearest neighbours, 3 x 3 actions (drifts along x1 and
    x2): AMGpi, FP64 and mixed."""
    import paper_1107_1653_amd as P
    from shapley_inputs import games
    g = games.point_cloud_game(1 << 18, seed=11)
    h = P.create_from(g)
    out = {}
    for name, prec in (("mixed", P.SHAPLEY_MIXED), ("fp64", P.SHAPLEY_FP64)):
        o = opts(P, args, prec)
        wall, lat, st, _ = timed(P, lambda: P.shapley_solve(h, o), args.steps, args.warmup)
        out[name] = {"value": g.n / (wall / args.steps), "ms_per_step": 1e3 * wall / args.steps,
                     "outer": st["outer"], "cycles": st["cycles_total"], "levels": st["levels"],
                     "op_complexity": st["op_complexity"], "residual": st["residual"]}
    P.shapley_game_destroy(h)
    line = record(args, out["mixed"]["value"], out["mixed"]["ms_per_step"], "f32+f64",
                  {"workload": f"point-cloud game n={g.n} (8 nearest neighbours, no grid), 3x3 actions, AMGpi to 1e-8"})
    line["extra"] = out
    return line


def iex1_line(args):
    """The paper's Isaacs example (Sec. 6.1, eq. (Iex1)) on 1025 x 1025 points
    with action sets around the continuous optimum (5 directions x 9 values of
    b per state), lambda = 0, to 1e-10 as in the paper's Table table1Iex1:
    AMGpi and FAMGpi (grids 33 ... 1025 points); errors against sin x1 sin x2."""
    import paper_1107_1653_amd as P
    from shapley_inputs import games
    pts = [33, 65, 129, 257, 513, 1025]
    t0 = time.perf_counter()
    levels = [games.iex1_local_game(p) for p in pts]
    g = levels[-1]
    log(f"[bench] iex1: generated {len(levels)} grids up to n={g.n} in {time.perf_counter() - t0:.1f}s")
    x1, x2 = games.grid_coords(g.grid)
    u = games.iex1_exact(x1, x2)
    out = {}
    h = P.create_from(g)
    for name, prec in (("amgpi_fp64", P.SHAPLEY_FP64), ("amgpi_mixed", P.SHAPLEY_MIXED)):
        o = P.shapley_default_opts(eps=1e-10, precision=prec, max_outer=5000, max_inner=5000, forcing=args.forcing,
                                   reuse_frac=args.reuse)
        wall, lat, st, _ = timed(P, lambda: P.shapley_solve(h, o), args.steps, args.warmup)
        v = P.shapley_get_value(h)
        out[name] = {"seconds": wall / args.steps, "outer": st["outer"], "inner": st["inner_total"],
                     "residual": st["residual"], "err_inf": float(np.max(np.abs(v - u))),
                     "err_l2": float(np.sqrt(np.mean((v - u) ** 2)))}
    P.shapley_game_destroy(h)
    H = P.shapley_game_create_hierarchy([P.create_from(x) for x in levels])
    of = P.shapley_default_opts(eps=1e-10, method=P.SHAPLEY_FAMGPI, c_fmg=0.1, max_outer=5000, max_inner=5000,
                                forcing=args.forcing, reuse_frac=args.reuse)
    wall, lat, st, _ = timed(P, lambda: P.shapley_solve(H, of), args.steps, args.warmup)
    v = P.shapley_get_value(H)
    out["famgpi_fp64"] = {"seconds": wall / args.steps, "outer": st["outer"], "residual": st["residual"],
                          "err_inf": float(np.max(np.abs(v - u))), "err_l2": float(np.sqrt(np.mean((v - u) ** 2)))}
    P.shapley_game_destroy(H)
    log(f"[bench] iex1: {out}")
    line = record(args, g.n / out["amgpi_fp64"]["seconds"], 1e3 * out["amgpi_fp64"]["seconds"], "f64",
                  {"workload": f"Isaacs example (Iex1), {pts[-1]}x{pts[-1]} points (n={g.n}), {g.m1}x{g.m2} actions "
                               "per state around the continuous optimum, AMGpi FP64 to 1e-10", "n": g.n})
    line["extra"] = out
    line["extra"]["paper"] = {"pi_lu_s": 277.0, "amgpi_s": 55.6, "famgpi_s": 18.5, "err_inf_1025": 4.13e-06,
                              "hardware": "serial C on an unstated CPU (context only)"}
    return line


def main() -> int:
    args = parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding across GPUs is not "
                                   "implemented)"}))
        return 2
    import torch  # noqa: F401  (device synchronisation around the timed regions)
    if args.calibrate_copy:
        calibration_kernel()
    if args.workload != "c3":
        fn = {"c0": c0_line, "c1": lambda a: c1_line(a, with_oracle=not a.no_cpu_baseline), "c2": c2_line,
              "c4": c4_line, "two_stopper": two_stopper_line, "general": general_line, "iex1": iex1_line}[args.workload]
        line = fn(args)
        print(json.dumps(line), flush=True)
        return 0
    line, gs, v_mixed = c3_line(args)
    extra = {}
    if not args.no_extra:
        extra["c2_isaacs3d_129"] = c2_line(args)
        extra["c1_obstacle_1025"] = c1_line(args, with_oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["error_vs_oracle"] = c3_cpu_baseline(args, gs, v_mixed)
        log(f"[bench] cpu baseline: {line['cpu_baseline']}")
    else:
        line["cpu_baseline"] = None
    line["extra"] = extra
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
