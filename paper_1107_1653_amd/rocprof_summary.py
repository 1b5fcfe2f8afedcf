"""Summaries of rocprofv3 output for this library's kernels.

    python -m paper_1107_1653_amd.rocprof_summary trace <results.db> [--top N] [--largest F,...]
        per-kernel calls / total / average duration from a --kernel-trace
        results database, and the same per probe family; with --largest,
        also each kernel of those families at its largest grid (for the
        streaming kernels: their launches on the finest level)
    python -m paper_1107_1653_amd.rocprof_summary traffic <fetch.csv> <write.csv> --out <json>
        HBM bytes per launch of each probe family from two --pmc runs
        (FETCH_SIZE, then WRITE_SIZE, output format csv) of a benchmark run
        made with --calibrate-copy: both counters are scaled by what they
        read for the calibration kernel, which reads and writes a known size;
        per family over all launches and over its launches at the largest
        grid (bytes_per_launch: the finest level, the roofline's launch set)

Probe families are the kernel groups the library can time with HIP events
(shapley_probe_enable): smooth, resid64, improve, resid, restrict, prolong,
rap (Galerkin product, both passes), interp, tail.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import sqlite3
import sys

CALIB_BYTES = 1 << 30  # must match the benchmark's calibration kernel

_FAMILIES = (  # (substring of the kernel name, family); first match wins
    ("k_resid64", "resid64"),
    ("k_smooth", "smooth"),
    ("k_improve", "improve"),
    ("k_resid<", "resid"),
    ("k_restrict", "restrict"),
    ("k_prolong", "prolong"),
    ("k_rap<", "rap"),
    ("k_rap_quad", "rap"),
    ("k_rap_thr", "rap"),
    ("k_rap_small", "rap"),
    ("k_rap_list", "rap"),
    ("k_drap_ap", "rap"),
    ("k_drap_ac", "rap"),
    ("k_drap_count", "rap"),
    ("k_drap_known", "rap"),
    ("k_interp", "interp"),
    ("k_tail<", "tail"),
)


# kernels that complete a launch of their family rather than start one: the
# Galerkin product of a large level is the wavefront kernel followed by the
# workgroup kernel over the rows it left (one probe launch, two kernels); the
# dense product of a small level starts with AP and continues with R (AP);
# interpolation redoes the rows its first pass deferred in a list kernel
_CONTINUATIONS = ("k_rap_list", "k_drap_ac", "k_drap_count", "k_drap_known", "k_interp_wave_list",
                  "k_interp_lds_list")


def starts_launch(name: str) -> bool:
    return not any(k in name for k in _CONTINUATIONS)


def is_refresh(name: str) -> bool:
    """Galerkin kernels of a refresh (known pattern: the kernels' mode 1),
    which recompute the changed rows only; the bench's probe claims no bytes
    for them, so the roofline's launch set is the full products."""
    n = short_name(name)
    if family_of(n) != "rap":
        return False
    lt = n.find("<")
    return "k_drap_known" in n or (lt >= 0 and n[lt + 1:lt + 2] == "1" and not n[lt + 2:lt + 3].isdigit()) \
        or n.endswith(", 1>")


def family_of(name: str):
    for key, fam in _FAMILIES:
        if key in name:
            return fam
    return None


def short_name(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def source_hash() -> str:
    """sha256 over the HIP sources and headers of the library (kernels and
    launch code): traffic figures are valid only for the sources measured."""
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(here)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(here, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def kernel_stats(db_path: str):
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    ni = cols.index("name") if "name" in cols else cols.index("kernel_name")
    si, ei = cols.index("start"), cols.index("end")
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in cur.execute("select * from kernels"):
        a = agg[short_name(r[ni])]
        a[0] += 1
        a[1] += (r[ei] - r[si]) / 1e3  # ns -> us
    db.close()
    return sorted(((k, c, t, t / c) for k, (c, t) in agg.items()), key=lambda x: -x[2])


def _grid_column(cols, axis):
    for name in (f"grid_{axis}", f"grid_size_{axis}"):
        if name in cols:
            return cols.index(name)
    return None


def largest_launches(db_path: str, families):
    """Per kernel of the given probe families: the launches at the largest
    grid the kernel ran with (kernel, grid size, launches, average us)."""
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    cols = [r[1] for r in cur.execute("pragma table_info(kernels)")]
    ni = cols.index("name") if "name" in cols else cols.index("kernel_name")
    si, ei = cols.index("start"), cols.index("end")
    gi = [g for g in (_grid_column(cols, a) for a in "xyz") if g is not None]
    if not gi:
        raise RuntimeError("no grid size column in the kernels table")
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: [0, 0.0]))
    for r in cur.execute("select * from kernels"):
        k = short_name(r[ni])
        if family_of(k) not in families:
            continue
        grid = 1
        for g in gi:
            grid *= max(int(r[g] or 1), 1)
        a = per[k][grid]
        a[0] += 1
        a[1] += (r[ei] - r[si]) / 1e3
    db.close()
    out = []
    for k, by_grid in per.items():
        grid = max(by_grid)
        c, t = by_grid[grid]
        out.append((k, grid, c, t / c))
    return sorted(out, key=lambda x: (family_of(x[0]), -x[1]))


def trace_summary(db_path: str, top: int = 25, largest=()) -> str:
    rows = kernel_stats(db_path)
    total = sum(r[2] for r in rows)
    lines = [f"total kernel time {total / 1e3:.2f} ms over {sum(r[1] for r in rows)} launches", "",
             "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for k, c, t, a in rows[:top]:
        lines.append(f"| `{k}` | {c} | {t / 1e3:.2f} | {a:.2f} | {100 * t / total:.1f}% |")
    fam = collections.defaultdict(lambda: [0, 0.0])
    for k, c, t, a in rows:
        f = family_of(k)
        if f:
            fam[f][0] += c if starts_launch(k) else 0
            fam[f][1] += t
    lines += ["", "| probe family | launches | total ms | avg us per launch |", "|---|---|---|---|"]
    for f, (c, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {f} | {c} | {t / 1e3:.2f} | {t / c:.2f} |")
    if largest:
        lines += ["", "| kernel at its largest grid | grid size | launches | avg us |", "|---|---|---|---|"]
        for k, g, c, a in largest_launches(db_path, largest):
            lines.append(f"| `{k}` | {g} | {c} | {a:.2f} |")
    return "\n".join(lines)


def _load_counter(path: str, counter: str):
    """(kernel name, grid size or 0, value in KiB) of every dispatch."""
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                grid = int(float(r.get("Grid_Size") or 0))
                out.append((r["Kernel_Name"], grid, float(r["Counter_Value"])))
    return out


def _per_family(rows, factor, largest, only=None):
    """Per family: launches and bytes.  largest: the dispatches of one kernel
    of the family at its largest grid -- the kernel whose dispatches there
    move the most bytes in all (a streaming kernel's finest level; the
    Galerkin product's and the interpolation's full setup of the finest
    level), the launch set of the bench's roofline."""
    top = collections.defaultdict(int)
    for k, g, _ in rows:
        top[short_name(k)] = max(top[short_name(k)], g)
    fam = collections.defaultdict(lambda: [0, 0.0])
    if not largest:
        for k, g, v in rows:
            f = family_of(k)
            if f:
                fam[f][0] += 1 if starts_launch(k) else 0
                fam[f][1] += factor * v * 1024.0
        return fam
    per_kernel = collections.defaultdict(lambda: [0, 0.0])  # at its largest grid
    for k, g, v in rows:
        n = short_name(k)
        if family_of(k) and starts_launch(k) and not is_refresh(k) and g == top[n]:
            per_kernel[n][0] += 1
            per_kernel[n][1] += factor * v * 1024.0
    best = {}
    for n, (c, b) in per_kernel.items():
        f = family_of(n)
        if only is not None:
            if only.get(f) == n:
                best[f] = (c, b, n)
        elif f not in best or b > best[f][1]:
            best[f] = (c, b, n)
    for f, (c, b, n) in best.items():
        fam[f] = [c, b, n]
    return fam


def traffic(fetch_csv: str, write_csv: str) -> dict:
    """HBM bytes per launch of each family, over all its launches and over
    its launches at the largest grid (the launch set the benchmark's roofline
    uses), both counters scaled by what they read for the calibration
    kernel."""
    fetch = _load_counter(fetch_csv, "FETCH_SIZE")
    write = _load_counter(write_csv, "WRITE_SIZE")
    cal_f = [v for k, _, v in fetch if "neg_kernel" in k]
    cal_w = [v for k, _, v in write if "neg_kernel" in k]
    if not cal_f or not cal_w:
        raise RuntimeError("no calibration kernel in the counter runs (use --calibrate-copy)")
    ff = CALIB_BYTES / (cal_f[0] * 1024.0)  # counters are in KiB
    fw = CALIB_BYTES / (cal_w[0] * 1024.0)
    out = {"calibration": {"bytes": CALIB_BYTES, "fetch_kib": cal_f[0], "write_kib": cal_w[0],
                           "fetch_factor": ff, "write_factor": fw},
           "families": {}}
    for largest in (False, True):
        fa = _per_family(fetch, ff, largest)
        # the same kernels for the writes as for the fetches
        wa = _per_family(write, fw, largest, {f: v[2] for f, v in fa.items()} if largest else None)
        for f in fa:
            n = max(fa[f][0], 1)
            fb, wb = fa[f][1] / n, wa[f][1] / n if f in wa else 0.0
            d = out["families"].setdefault(f, {})
            if largest:
                d.update({"largest_launches": fa[f][0], "kernel": fa[f][2], "fetch_bytes_per_launch": fb,
                          "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb})
            else:
                d.update({"launches": fa[f][0], "all_fetch_bytes_per_launch": fb,
                          "all_write_bytes_per_launch": wb, "all_bytes_per_launch": fb + wb})
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=25)
    t.add_argument("--largest", default="", help="comma-separated probe families")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_csv")
    c.add_argument("write_csv")
    c.add_argument("--out", required=True)
    c.add_argument("--command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        fams = tuple(f for f in a.largest.split(",") if f)
        print(trace_summary(a.db, a.top, fams))
    else:
        d = traffic(a.fetch_csv, a.write_csv)
        d["source_sha256"] = source_hash()
        d["command"] = a.command
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
        print(json.dumps(d["families"], indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
