"""The C-ABI library loads and exports every function include/shapley.h
declares; option and statistics structs match the header (no GPU calls)."""
import ctypes
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shapley.h")
LIB = os.path.join(ROOT, "paper_1107_1653_amd", "libshapley.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shapley_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("shapley_game_create", "shapley_game_create_hierarchy", "shapley_solve",
                     "shapley_get_value", "shapley_get_policy", "shapley_game_destroy",
                     "shapley_solve_batch", "shapley_server_create", "shapley_server_submit",
                     "shapley_server_wait", "shapley_server_poll", "shapley_server_destroy",
                     "shapley_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    import paper_1107_1653_amd as P
    assert sorted(P.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_default_options_match_header_documentation():
    import paper_1107_1653_amd as P
    o = P.shapley_default_opts()
    assert o.eps == 0.0 and o.precision == P.SHAPLEY_FP64 and o.method == P.SHAPLEY_AMGPI
    assert o.c_fmg == 1e-2 and o.max_cycles == 200 and o.lin_rtol == 1e-14 and o.tie_rtol == 1e-12
    assert o.nu1 == 2 and o.nu2 == 2 and o.omega == 0.8 and o.coarse_max == 64
    assert o.reuse_frac == 0.5 and o.forcing == 0.0
    assert o.smoother == P.SHAPLEY_SMOOTH_JACOBI and o.gamma == 1 and o.graph == 1
    # the struct layout in the binding equals the C layout: the C side wrote
    # the last field (graph) where the binding reads it
    assert ctypes.sizeof(P.shapley_solve_opts) == (P.shapley_solve_opts.graph.offset + 4 + 7) // 8 * 8


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_probe_arguments_are_checked():
    # no launches probed: nothing touches a device
    import paper_1107_1653_amd as P
    P.shapley_probe_enable("smooth", True)
    assert P.shapley_probe_read_large("smooth", 0.5) == dict(launches=0, ms=0.0, bytes=0.0)
    for frac in (0.0, -1.0, 1.5, float("nan")):
        with pytest.raises(P.ShapleyError):
            P.shapley_probe_read_large("smooth", frac)
    P.shapley_probe_enable("smooth", False)
    lib = ctypes.CDLL(LIB)
    n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    assert lib.shapley_probe_read_large(99, ctypes.c_double(0.5), ctypes.byref(n), ctypes.byref(ms),
                                        ctypes.byref(b)) == P.SHAPLEY_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_lane_control_arguments():
    # the setting only takes effect at later setups: no device call here
    import paper_1107_1653_amd as P
    for bad in (3, 8, 16, -1):
        with pytest.raises(P.ShapleyError):
            P.shapley_tune_lanes(bad)
    for ok in (1, 2, 4, 0):
        P.shapley_tune_lanes(ok)
    for bad in (2, 8, 32, -2):
        with pytest.raises(P.ShapleyError):
            P.shapley_tune_galerkin(bad)
    for ok in (0, 1, 4, -1):
        P.shapley_tune_galerkin(ok)
    for bad in (1, 2, 8, -2):
        with pytest.raises(P.ShapleyError):
            P.shapley_tune_interp(bad)
    for ok in (0, 4, -1):
        P.shapley_tune_interp(ok)
    for bad in (1, 4, -2):
        with pytest.raises(P.ShapleyError):
            P.shapley_tune_dense(bad)
    for ok in (0, -1):
        P.shapley_tune_dense(ok)
    with pytest.raises(P.ShapleyError):
        P.shapley_debug_fail_alloc(-1)
    P.shapley_debug_fail_alloc(0)


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in json.loads(out.stdout.strip())["error"]
