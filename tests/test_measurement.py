"""Host side of the measurement path (CPU): the rocprofv3 summaries the
profiles are made with, the bench's counter-traffic lookup and its one-GPU
contract.  No GPU is used."""
import csv
import json
import os
import sqlite3
import subprocess
import sys

import pytest

from paper_1107_1653_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for row in rows:
            name, value = row[0], row[-1]
            grid = row[1] if len(row) == 3 else 256
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_is_scaled_by_the_calibration_kernel(tmp_path):
    cal = rs.CALIB_BYTES
    # the calibration kernel reads as FETCH_SIZE half of what it moves and
    # writes its full size: factors 2 and 1
    fetch = [("void at::native::neg_kernel(...)", cal / 2 / 1024),
             ("void shp::k_smooth<double, 4>(...)", 1000.0),
             ("void shp::k_smooth<double, 1>(...)", 3000.0),
             ("void shp::k_rap_small<0>(...)", 500.0),
             ("void shp::k_rap_list<128, 0>(...)", 100.0),  # completes the previous launch
             ("shp::k_drap_ap<true, 1024>(...)", 40.0),
             ("shp::k_drap_ac(...)", 20.0),
             ("shp::k_drap_count(...)", 4.0),
             ("shp::k_scan_block(...)", 7.0)]                # no family
    write = [("void at::native::neg_kernel(...)", cal / 1024),
             ("void shp::k_smooth<double, 4>(...)", 10.0),
             ("void shp::k_smooth<double, 1>(...)", 30.0),
             ("void shp::k_rap_small<0>(...)", 50.0),
             ("void shp::k_rap_list<128, 0>(...)", 10.0),
             ("shp::k_drap_ap<true, 1024>(...)", 4.0),
             ("shp::k_drap_ac(...)", 2.0),
             ("shp::k_drap_count(...)", 0.0),
             ("shp::k_scan_block(...)", 1.0)]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fcsv, "FETCH_SIZE", fetch)
    write_counters(wcsv, "WRITE_SIZE", write)
    d = rs.traffic(str(fcsv), str(wcsv))
    assert d["calibration"]["fetch_factor"] == pytest.approx(2.0)
    assert d["calibration"]["write_factor"] == pytest.approx(1.0)
    sm = d["families"]["smooth"]
    assert sm["launches"] == 2
    assert sm["all_fetch_bytes_per_launch"] == pytest.approx(2.0 * 4000.0 * 1024 / 2)
    assert sm["all_write_bytes_per_launch"] == pytest.approx(40.0 * 1024 / 2)
    rap = d["families"]["rap"]
    # two launches (the row-wise and the dense product); the list kernel and
    # the dense product's later kernels continue a launch
    assert rap["launches"] == 2
    assert rap["all_fetch_bytes_per_launch"] == pytest.approx(2.0 * 664.0 * 1024 / 2)
    assert rap["all_bytes_per_launch"] == pytest.approx(rap["all_fetch_bytes_per_launch"] + 66.0 * 1024 / 2)
    assert "scan" not in d["families"]


def test_traffic_of_the_largest_launches(tmp_path):
    """bytes_per_launch covers the launches of one kernel of the family at its
    largest grid -- the kernel moving the most bytes there in all (the
    finest level) --, the launch set of the benchmark's roofline; a
    refresh's Galerkin kernels are left out of it."""
    cal = rs.CALIB_BYTES
    fetch = [("void at::native::neg_kernel(...)", 1, cal / 2 / 1024),
             ("shp::k_smooth<float, 4>(...)", 4 << 20, 3000.0),
             ("shp::k_smooth<float, 4>(...)", 4 << 20, 5000.0),
             ("shp::k_smooth<float, 4>(...)", 1 << 20, 100.0),
             ("shp::k_smooth<float, 1>(...)", 1 << 16, 10.0)]
    write = [("void at::native::neg_kernel(...)", 1, cal / 1024),
             ("shp::k_smooth<float, 4>(...)", 4 << 20, 30.0),
             ("shp::k_smooth<float, 4>(...)", 4 << 20, 50.0),
             ("shp::k_smooth<float, 4>(...)", 1 << 20, 1.0),
             ("shp::k_smooth<float, 1>(...)", 1 << 16, 1.0)]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fcsv, "FETCH_SIZE", fetch)
    write_counters(wcsv, "WRITE_SIZE", write)
    sm = rs.traffic(str(fcsv), str(wcsv))["families"]["smooth"]
    assert sm["launches"] == 4
    # the kernel moving the most at its largest grid: the two big
    # k_smooth<float, 4> dispatches
    assert sm["largest_launches"] == 2 and sm["kernel"] == "shp::k_smooth<float, 4>"
    assert sm["fetch_bytes_per_launch"] == pytest.approx(2.0 * 8000.0 * 1024 / 2)
    assert sm["write_bytes_per_launch"] == pytest.approx(80.0 * 1024 / 2)


def test_refresh_kernels_are_not_the_roofline_launches():
    assert rs.is_refresh("void shp::k_rap_small<1>(int)")
    assert rs.is_refresh("void shp::k_rap_quad<1, 32>(int)")
    assert rs.is_refresh("void shp::k_rap_list<128, 1>(int)")
    assert rs.is_refresh("shp::k_drap_known(int)")
    assert not rs.is_refresh("void shp::k_rap_quad<0, 32>(int)")
    assert not rs.is_refresh("void shp::k_rap_small<0>(int)")
    assert not rs.is_refresh("void shp::k_rap_list<128, 0>(int)")
    assert not rs.is_refresh("void shp::k_smooth<float, 1>(int)")


def test_traffic_needs_the_calibration_kernel(tmp_path):
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(fcsv, "FETCH_SIZE", [("shp::k_improve(...)", 1.0)])
    write_counters(wcsv, "WRITE_SIZE", [("shp::k_improve(...)", 1.0)])
    with pytest.raises(RuntimeError):
        rs.traffic(str(fcsv), str(wcsv))


def test_trace_summary_counts_launches_per_family(tmp_path):
    db = tmp_path / "t.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer, grid_size_x integer, "
                "grid_size_y integer, grid_size_z integer)")
    rows = [("void shp::k_tail<double>(int)", 0, 20000), ("void shp::k_tail<double>(int)", 30000, 70000),
            ("void shp::k_rap_small<1>(int)", 0, 5000), ("void shp::k_rap_list<128, 1>(int)", 6000, 8000),
            ("shp::k_drap_ap<false, 2048>(int)", 0, 1000), ("shp::k_drap_known(int)", 1000, 4000)]
    rows = [r + (256, 1, 1) for r in rows]
    # a streaming kernel on two levels: its largest grid is the finest level
    rows += [("void shp::k_smooth<double, 4>(int)", 0, 30000, 4 << 20, 1, 1),
             ("void shp::k_smooth<double, 4>(int)", 0, 34000, 4 << 20, 1, 1),
             ("void shp::k_smooth<double, 4>(int)", 0, 9000, 1 << 20, 1, 1),
             ("void shp::k_smooth<double, 16>(int)", 0, 2000, 1 << 18, 1, 1)]
    con.executemany("insert into kernels values (?, ?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    stats = {k: (c, t) for k, c, t, _ in rs.kernel_stats(str(db))}
    assert stats["shp::k_tail<double>"] == (2, pytest.approx(60.0))
    text = rs.trace_summary(str(db))
    fam = {}
    for line in text.splitlines():
        parts = [p.strip() for p in line.strip("|").split("|")]
        if len(parts) == 4 and parts[0] in ("tail", "rap"):
            fam[parts[0]] = (int(parts[1]), float(parts[2]), float(parts[3]))
    assert fam["tail"] == (2, pytest.approx(0.06), pytest.approx(30.0))
    # rap: the wavefront kernel and the dense AP start launches (2); the list
    # kernel and the dense R(AP) pass continue them; 11 us in all
    assert fam["rap"] == (2, pytest.approx(0.011, abs=0.005), pytest.approx(5.5))  # total printed to 0.01 ms
    big = {k: (g, c, a) for k, g, c, a in rs.largest_launches(str(db), ("smooth",))}
    assert big == {"shp::k_smooth<double, 4>": (4 << 20, 2, pytest.approx(32.0)),
                   "shp::k_smooth<double, 16>": (1 << 18, 1, pytest.approx(2.0))}
    assert "| `shp::k_smooth<double, 4>` | 4194304 | 2 | 32.00 |" in rs.trace_summary(str(db), largest=("smooth",))


def test_bench_reports_no_traffic_for_changed_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    (tmp_path / "profiles").mkdir()
    f = tmp_path / "profiles" / "traffic_c3.json"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    f.write_text(json.dumps({"source_sha256": "0" * 64, "families": {"rap": {"bytes_per_launch": 1.0}}}))
    value, why = bench.traffic_for("c3", "rap")
    assert value is None and "changed" in why
    f.write_text(json.dumps({"source_sha256": rs.source_hash(), "families": {"rap": {"bytes_per_launch": 5.0}}}))
    value, why = bench.traffic_for("c3", "rap")
    assert value == 5.0
    value, why = bench.traffic_for("c3", "tail")
    assert value is None
    value, why = bench.traffic_for("c2", "rap")
    assert value is None and "no counter" in why


def test_bench_roofline_object():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.roofline("c9", "smooth", {"launches": 4, "ms": 0.2, "bytes": 4e9})
    # 1e9 bytes per launch in 50 us: 20000 GB/s
    assert r["achieved"] == pytest.approx(2e4) and r["frac"] == pytest.approx(2.5)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert bench.roofline("c9", "rap", {"launches": 1, "ms": 1.0, "bytes": 1.0})["bound"] == "latency"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
