"""Oracle solves of benchmark games in worker processes -- TEST
INFRASTRUCTURE, like the rest of this package: only the tests, the smoke
check and the benchmark's CPU-baseline leg run it.

A job is (name, recipe, args, eps): the worker rebuilds the game from its
seeded recipe, runs the FP64 oracle (policy iteration, or FAMGpi for the
obstacle grids) to the Shapley residual eps (0: the fixed point, no policy
improves) and writes the value, both strategies and the tie flags to
<out>/<name>.npz.  Workers are separate Python processes started with
subprocess (no GPU, one BLAS thread each), so a GPU process can run them
beside its own work.

    python -m oracle.jobs <jobs.json> <out_dir>     # one worker
"""
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _build(recipe, args, eps):
    """Returns (game whose solution is compared, oracle result)."""
    from . import shapley_oracle as orc
    from shapley_inputs import configs
    if recipe == "c3":                       # (k, side, lam)
        g = configs.c3_game(*args)
        return g, orc.policy_iteration(g, eps=eps)
    if recipe == "c4_isaacs":                # (side, lam, seed)
        side, lam, seed = args
        g = configs.c4_game(0, side, lam, seed)
        return g, orc.policy_iteration(g, eps=eps)
    if recipe == "c4_obstacle":              # (side, seed, lam): FAMGpi on its grids
        side, seed, lam = args
        lv = configs.obstacle_levels_for_side(side, seed, lam)
        a0 = np.zeros(lv[0].n, np.int32)
        return lv[-1], orc.famg_pi(lv, eps=eps, c=1e-2, alpha0=a0, beta0=a0)[-1]
    if recipe == "c1":                       # (points, coarsest_points)
        lv = configs.c1_levels(points=args[0], coarsest_points=args[1])
        a0 = np.zeros(lv[0].n, np.int32)
        return lv[-1], orc.famg_pi(lv, eps=eps, c=1e-2, alpha0=a0, beta0=a0)[-1]
    raise ValueError(recipe)


def _work(jobs_path, out_dir):
    from . import shapley_oracle as orc
    with open(jobs_path) as f:
        jobs = json.load(f)
    for name, recipe, args, eps in jobs:
        t = time.perf_counter()
        g, res = _build(recipe, args, eps)
        tied = orc.tied_states(g, res.v, res.alpha)
        np.savez(os.path.join(out_dir, name + ".tmp.npz"), v=res.v, alpha=res.alpha, beta=res.beta, tied=tied,
                 seconds=time.perf_counter() - t, converged=res.converged)
        os.replace(os.path.join(out_dir, name + ".tmp.npz"), os.path.join(out_dir, name + ".npz"))


class Jobs:
    """Oracle jobs (name, recipe, args, eps) running in up to `workers`
    processes, longest first (cost: estimated seconds of a job)."""

    def __init__(self, jobs, cost=None, workers=None):
        self.dir = tempfile.mkdtemp(prefix="oracle_jobs_")
        workers = workers or min(16, os.cpu_count() or 1)
        order = sorted(jobs, key=lambda j: -(cost(j) if cost else 1.0))
        chunks = [[] for _ in range(min(workers, max(len(order), 1)))]
        load = [0.0] * len(chunks)
        for j in order:                      # greedy balance by estimated cost
            k = load.index(min(load))
            chunks[k].append(j)
            load[k] += cost(j) if cost else 1.0
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = "1"
        env["HIP_VISIBLE_DEVICES"] = ""
        env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
        self.names = [j[0] for j in jobs]
        self.workers = sum(1 for ch in chunks if ch)
        self.procs = []
        for i, ch in enumerate(chunks):
            if not ch:
                continue
            path = os.path.join(self.dir, f"jobs{i}.json")
            with open(path, "w") as f:
                json.dump(ch, f)
            self.procs.append(subprocess.Popen([sys.executable, "-m", "oracle.jobs", path, self.dir], env=env,
                                               cwd=ROOT, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
        self.t_start = time.perf_counter()
        self.t_end = None

    def wait(self, timeout=600.0, log=None):
        """Dict name -> dict(v, alpha, beta, tied, seconds); raises if a worker failed."""
        t0 = time.perf_counter()
        last = -1
        while any(p.poll() is None for p in self.procs):
            done = sum(os.path.exists(os.path.join(self.dir, n + ".npz")) for n in self.names)
            if log and done != last:
                log(f"  oracle jobs: {done}/{len(self.names)} done after {time.perf_counter() - t0:.0f} s")
                last = done
            if time.perf_counter() - t0 > timeout:
                for p in self.procs:
                    p.kill()
                raise TimeoutError("oracle jobs did not finish")
            time.sleep(0.5)
        if self.t_end is None:
            self.t_end = time.perf_counter()
        for p in self.procs:
            if p.returncode != 0:
                raise RuntimeError("oracle worker failed: " + p.stderr.read().decode()[-2000:])
        out = {}
        for n in self.names:
            with np.load(os.path.join(self.dir, n + ".npz")) as d:
                out[n] = {k: d[k] for k in d.files}
        return out


    @property
    def seconds(self):
        """Wall time from the start of the workers to the end of the last one."""
        return (self.t_end or time.perf_counter()) - self.t_start


if __name__ == "__main__":
    _work(sys.argv[1], sys.argv[2])
