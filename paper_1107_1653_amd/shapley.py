"""Thin ctypes binding of libshapley (argument marshalling only).

The functions keep the names of the C ABI declared in include/shapley.h.
All computation happens in the HIP library; if the library cannot be loaded
every call raises.  PyTorch is only used, when the caller passes tensors or
streams, to obtain device pointers and stream handles.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libshapley.so")

SHAPLEY_OK = 0
SHAPLEY_EINVAL = 1
SHAPLEY_ENOMEM = 2
SHAPLEY_ENOCONV = 3
SHAPLEY_EDEVICE = 4
SHAPLEY_EAGAIN = 5
SHAPLEY_FP64 = 0
SHAPLEY_MIXED = 1
SHAPLEY_AMGPI = 0
SHAPLEY_FAMGPI = 1
SHAPLEY_HOST_PTRS = 0
SHAPLEY_DEVICE_PTRS = 1
SHAPLEY_SMOOTH_JACOBI = 0
SHAPLEY_SMOOTH_L1 = 1
SHAPLEY_SMOOTH_CF = 2

EXPORTED = [
    "shapley_last_error", "shapley_default_opts", "shapley_game_create",
    "shapley_game_create_hierarchy", "shapley_solve", "shapley_get_value", "shapley_get_policy",
    "shapley_apply_operator", "shapley_apply_operator_noalloc", "shapley_game_info", "shapley_game_bytes", "shapley_hierarchy_level",
    "shapley_game_destroy",
    "shapley_solve_batch", "shapley_server_create", "shapley_server_submit", "shapley_server_wait",
    "shapley_server_poll", "shapley_server_step", "shapley_server_destroy", "shapley_server_info",
    "shapley_probe_enable", "shapley_probe_read", "shapley_probe_read_large", "shapley_tune_lanes",
    "shapley_tune_galerkin", "shapley_tune_interp", "shapley_tune_stencil", "shapley_debug_fail_alloc",
    "shapley_tune_dense", "shapley_coarse_inverse",
]
PROBE = dict(smooth=0, resid64=1, improve=2, resid=3, restrict=4, prolong=5, rap=6, interp=7, tail=8)


class ShapleyError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libshapley error {code}: {msg}")
        self.code = code


class shapley_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("s", C.c_int32), ("bvals", C.POINTER(C.c_double))]


class shapley_solve_opts(C.Structure):
    _fields_ = [
        ("eps", C.c_double), ("precision", C.c_int32), ("method", C.c_int32), ("c_fmg", C.c_double),
        ("alpha0", C.POINTER(C.c_int32)), ("beta0", C.POINTER(C.c_int32)), ("v0", C.POINTER(C.c_double)),
        ("max_outer", C.c_int32), ("max_inner", C.c_int32), ("max_cycles", C.c_int32),
        ("lin_rtol", C.c_double), ("lin_atol", C.c_double), ("tie_rtol", C.c_double),
        ("theta", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32), ("omega", C.c_double),
        ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("verbose", C.c_int32),
        ("stream", C.c_void_p), ("reuse_frac", C.c_double), ("forcing", C.c_double),
        ("smoother", C.c_int32), ("gamma", C.c_int32), ("graph", C.c_int32),
    ]


class shapley_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int32), ("active", C.c_int32), ("cohorts", C.c_int32), ("reserved", C.c_int32),
                ("budget_used", C.c_size_t), ("budget", C.c_size_t)]


class shapley_level_info(C.Structure):
    _fields_ = [("levels", C.c_int32), ("pw", C.c_int32), ("n", C.c_int64), ("nnz", C.c_int64),
                ("nc", C.c_int64)]


class shapley_stats(C.Structure):
    _fields_ = [
        ("outer", C.c_int32), ("inner_total", C.c_int32), ("cycles_total", C.c_int32),
        ("levels", C.c_int32), ("converged", C.c_int32), ("fmg_levels", C.c_int32),
        ("residual", C.c_double), ("residual_l2", C.c_double), ("seconds", C.c_double),
        ("setup_seconds", C.c_double), ("cycle_seconds", C.c_double), ("improve_seconds", C.c_double),
        ("op_complexity", C.c_double), ("grid_complexity", C.c_double),
        ("inner_per_outer", C.c_int32 * 64),
        ("setups_full", C.c_int32), ("setups_refresh", C.c_int32), ("value_steps", C.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "inner_per_outer"}
        d["inner_per_outer"] = [int(x) for x in self.inner_per_outer[: min(self.outer, 64)]]
        return d


_lib_handle = None


def lib() -> C.CDLL:
    """Loads libshapley.so; raises if it is missing (there is no fallback)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1107_1653_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname.  Loaded
        # first, it is the one the library binds to, so that PyTorch's
        # streams and device pointers can be handed to the library; loaded
        # second, the process would hold two runtimes that do not share them.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.shapley_last_error.restype = C.c_char_p
        L.shapley_default_opts.argtypes = [C.POINTER(shapley_solve_opts)]
        L.shapley_game_create.argtypes = [C.POINTER(P), C.c_int64, C.c_int32, C.c_int32, P, P, P, P,
                                          C.c_double, P, C.POINTER(shapley_grid), C.c_uint32, P]
        L.shapley_game_create_hierarchy.argtypes = [C.POINTER(P), C.c_int32, C.POINTER(P)]
        L.shapley_solve.argtypes = [P, C.POINTER(shapley_solve_opts), C.POINTER(shapley_stats)]
        L.shapley_get_value.argtypes = [P, P, C.c_int32]
        L.shapley_get_policy.argtypes = [P, P, P, P]
        L.shapley_apply_operator.argtypes = [P, P, P, P, P]
        L.shapley_apply_operator_noalloc.argtypes = [P, P, P, P, P, P, P]
        L.shapley_game_info.argtypes = [P, P, P, P]
        L.shapley_game_bytes.argtypes = [P, C.POINTER(C.c_size_t)]
        L.shapley_hierarchy_level.argtypes = [P, C.c_int32, C.POINTER(shapley_level_info), P, P, P, P, P]
        L.shapley_game_destroy.argtypes = [P]
        L.shapley_game_destroy.restype = None
        L.shapley_solve_batch.argtypes = [C.POINTER(P), C.c_int32, C.POINTER(shapley_solve_opts),
                                          C.POINTER(shapley_stats)]
        L.shapley_server_create.argtypes = [C.POINTER(P), C.c_size_t, P]
        L.shapley_server_submit.argtypes = [P, P, C.POINTER(shapley_solve_opts), C.POINTER(C.c_uint64)]
        L.shapley_server_wait.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(shapley_stats)]
        L.shapley_server_poll.argtypes = [P, C.c_uint64, C.POINTER(shapley_stats)]
        L.shapley_server_step.argtypes = [P, C.POINTER(C.c_int32)]
        L.shapley_server_info.argtypes = [P, C.POINTER(shapley_server_stats)]
        L.shapley_server_destroy.argtypes = [P]
        L.shapley_server_destroy.restype = None
        L.shapley_probe_enable.argtypes = [C.c_int32, C.c_int32]
        L.shapley_probe_read.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]
        L.shapley_probe_read_large.argtypes = [C.c_int32, C.c_double, C.POINTER(C.c_int64),
                                               C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.shapley_tune_lanes.argtypes = [C.c_int32]
        L.shapley_tune_galerkin.argtypes = [C.c_int32]
        L.shapley_tune_interp.argtypes = [C.c_int32]
        L.shapley_tune_stencil.argtypes = [C.c_int32]
        L.shapley_debug_fail_alloc.argtypes = [C.c_int64]
        L.shapley_tune_dense.argtypes = [C.c_int32]
        L.shapley_coarse_inverse.argtypes = [P, P, C.c_int32, P]
        _lib_handle = L
    return _lib_handle


def _check(rc: int, allow=(SHAPLEY_OK,)) -> int:
    if rc not in allow:
        raise ShapleyError(rc, shapley_last_error())
    return rc


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
# same-name wrappers
# ---------------------------------------------------------------------------

def shapley_last_error() -> str:
    return lib().shapley_last_error().decode()


def shapley_default_opts(**kw) -> shapley_solve_opts:
    o = shapley_solve_opts()
    lib().shapley_default_opts(C.byref(o))
    _keep = []
    for k, v in kw.items():
        if k in ("alpha0", "beta0"):
            arr = np.ascontiguousarray(v, dtype=np.int32)
            _keep.append(arr)
            setattr(o, k, arr.ctypes.data_as(C.POINTER(C.c_int32)))
        elif k == "v0":
            arr = np.ascontiguousarray(v, dtype=np.float64)
            _keep.append(arr)
            setattr(o, k, arr.ctypes.data_as(C.POINTER(C.c_double)))
        elif k == "stream":
            setattr(o, k, None if v is None else int(getattr(v, "cuda_stream", v)))
        else:
            setattr(o, k, v)
    o._keep = _keep  # keep warm-start arrays alive with the struct
    return o


def _dev_ptr(t, dtype):
    """Device pointer of a contiguous torch tensor of the given torch dtype."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype):
        raise ValueError(f"expected a contiguous device tensor of {dtype}")
    return C.c_void_p(t.data_ptr())


def shapley_game_create(n, m1, m2, row_ptr, col, w, r, mu, valid=None, grid=None, flags=0, stream=None):
    if flags == SHAPLEY_DEVICE_PTRS:
        return _create_device(n, m1, m2, row_ptr, col, w, r, mu, valid, grid, stream)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    vv = None if valid is None else np.ascontiguousarray(valid, dtype=np.uint8)
    gp = None
    bv = None
    if grid is not None:
        dim, s, bvals = grid
        gs = shapley_grid()
        gs.dim, gs.s = int(dim), int(s)
        if bvals is not None:
            bv = np.ascontiguousarray(bvals, dtype=np.float64)
            gs.bvals = bv.ctypes.data_as(C.POINTER(C.c_double))
        gp = C.byref(gs)
    h = C.c_void_p()
    st = None if stream is None else C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    _check(lib().shapley_game_create(C.byref(h), int(n), int(m1), int(m2), _ptr(rp), _ptr(ci), _ptr(ww),
                                     _ptr(rr), float(mu), _ptr(vv), gp, int(flags), st))
    return h


def _create_device(n, m1, m2, row_ptr, col, w, r, mu, valid, grid, stream):
    """Create from torch device tensors (int64 row_ptr, int32 col, float64 w and
    r, uint8 valid, float64 grid bvals): only their pointers are passed."""
    import torch
    gp = None
    keep = []
    if grid is not None:
        dim, s, bvals = grid
        gs = shapley_grid()
        gs.dim, gs.s = int(dim), int(s)
        if bvals is not None:
            keep.append(bvals)
            gs.bvals = C.cast(_dev_ptr(bvals, torch.float64), C.POINTER(C.c_double))
        gp = C.byref(gs)
    h = C.c_void_p()
    st = None if stream is None else C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    _check(lib().shapley_game_create(C.byref(h), int(n), int(m1), int(m2), _dev_ptr(row_ptr, torch.int64),
                                     _dev_ptr(col, torch.int32), _dev_ptr(w, torch.float64),
                                     _dev_ptr(r, torch.float64), float(mu), _dev_ptr(valid, torch.uint8), gp,
                                     SHAPLEY_DEVICE_PTRS, st))
    return h


def shapley_game_create_hierarchy(levels: Sequence) -> C.c_void_p:
    arr = (C.c_void_p * len(levels))(*[lv.value if isinstance(lv, C.c_void_p) else lv for lv in levels])
    h = C.c_void_p()
    _check(lib().shapley_game_create_hierarchy(C.byref(h), len(levels), arr))
    return h


def shapley_solve(g, opts: Optional[shapley_solve_opts] = None, allow_noconv: bool = False) -> dict:
    st = shapley_stats()
    allow = (SHAPLEY_OK, SHAPLEY_ENOCONV) if allow_noconv else (SHAPLEY_OK,)
    rc = _check(lib().shapley_solve(g, None if opts is None else C.byref(opts), C.byref(st)), allow)
    d = st.as_dict()
    d["rc"] = rc
    return d


def shapley_solve_batch(games: Sequence, opts: Optional[shapley_solve_opts] = None,
                        allow_noconv: bool = False) -> list:
    arr = (C.c_void_p * len(games))(*[g.value for g in games])
    st = (shapley_stats * len(games))()
    allow = (SHAPLEY_OK, SHAPLEY_ENOCONV) if allow_noconv else (SHAPLEY_OK,)
    _check(lib().shapley_solve_batch(arr, len(games), None if opts is None else C.byref(opts), st), allow)
    return [s.as_dict() for s in st]


def shapley_apply_operator_noalloc(g, v, F, alpha, beta, res=None, stream=None) -> None:
    """Torch device tensors (float64 v, F, res; int32 alpha, beta) in and out;
    queued on `stream` (a torch stream or handle; None: the handle's)."""
    import torch
    ptr = lambda t, dt: None if t is None else _dev_ptr(t, dt)
    st = None if stream is None else C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    _check(lib().shapley_apply_operator_noalloc(g, ptr(v, torch.float64), ptr(F, torch.float64),
                                                ptr(alpha, torch.int32), ptr(beta, torch.int32),
                                                ptr(res, torch.float64), st))


def shapley_game_info(g):
    n, m1, m2 = C.c_int64(), C.c_int32(), C.c_int32()
    _check(lib().shapley_game_info(g, C.byref(n), C.byref(m1), C.byref(m2)))
    return n.value, m1.value, m2.value


def shapley_get_value(g, out=None):
    """Host copy of the value, or into a device tensor `out` (torch)."""
    if out is not None and hasattr(out, "data_ptr"):
        _check(lib().shapley_get_value(g, C.c_void_p(out.data_ptr()), 1))
        return out
    n, _, _ = shapley_game_info(g)
    v = np.empty(n, dtype=np.float64)
    _check(lib().shapley_get_value(g, _ptr(v), 0))
    return v


def shapley_get_policy(g, beta_all: bool = False):
    n, m1, _ = shapley_game_info(g)
    a = np.empty(n, dtype=np.int32)
    b = np.empty(n, dtype=np.int32)
    ba = np.empty(n * m1, dtype=np.int32) if beta_all else None
    _check(lib().shapley_get_policy(g, _ptr(a), _ptr(b), _ptr(ba)))
    return (a, b, ba.reshape(n, m1)) if beta_all else (a, b)


def shapley_apply_operator(g, v):
    n, _, _ = shapley_game_info(g)
    vv = np.ascontiguousarray(v, dtype=np.float64)
    F = np.empty(n)
    a = np.empty(n, dtype=np.int32)
    b = np.empty(n, dtype=np.int32)
    _check(lib().shapley_apply_operator(g, _ptr(vv), _ptr(F), _ptr(a), _ptr(b)))
    return F, a, b


def shapley_hierarchy_level(g, level: int, sizes_only: bool = False) -> dict:
    """Level `level` of the AMG hierarchy of g's last solve: A (CSR arrays
    rp, ci, a), P (pc, pv of shape (n, pw), only when nc > 0) and the sizes
    (the sizes alone with sizes_only)."""
    info = shapley_level_info()
    _check(lib().shapley_hierarchy_level(g, int(level), C.byref(info), None, None, None, None, None))
    n, nnz, nc, pw = info.n, info.nnz, info.nc, info.pw
    if sizes_only:
        return {"levels": info.levels, "n": n, "nnz": nnz, "nc": nc, "pw": pw}
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(max(nnz, 1), np.int32)
    a = np.empty(max(nnz, 1), np.float64)
    pc = np.empty((n, pw), np.int32) if nc else None
    pv = np.empty((n, pw), np.float64) if nc else None
    _check(lib().shapley_hierarchy_level(g, int(level), C.byref(info), _ptr(rp), _ptr(ci), _ptr(a), _ptr(pc),
                                         _ptr(pv)))
    return {"levels": info.levels, "n": n, "nnz": nnz, "nc": nc, "pw": pw, "rp": rp, "ci": ci[:nnz],
            "a": a[:nnz], "pc": pc, "pv": pv}


def shapley_game_bytes(g) -> int:
    b = C.c_size_t()
    _check(lib().shapley_game_bytes(g, C.byref(b)))
    return b.value


def shapley_game_destroy(g) -> None:
    lib().shapley_game_destroy(g)


def shapley_server_create(hbm_budget: int, stream=None):
    h = C.c_void_p()
    st = None if stream is None else C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    _check(lib().shapley_server_create(C.byref(h), int(hbm_budget), st))
    return h


def shapley_server_submit(srv, g, opts: Optional[shapley_solve_opts] = None) -> int:
    t = C.c_uint64()
    _check(lib().shapley_server_submit(srv, g, None if opts is None else C.byref(opts), C.byref(t)))
    return t.value


def shapley_server_step(srv) -> int:
    a = C.c_int32()
    _check(lib().shapley_server_step(srv, C.byref(a)))
    return a.value


def shapley_server_poll(srv, ticket: int):
    st = shapley_stats()
    rc = lib().shapley_server_poll(srv, C.c_uint64(ticket), C.byref(st))
    if rc == SHAPLEY_EAGAIN:
        return None
    _check(rc, (SHAPLEY_OK, SHAPLEY_ENOCONV))
    d = st.as_dict()
    d["rc"] = rc
    return d


def shapley_server_wait(srv, ticket: int, max_steps: int = 0):
    st = shapley_stats()
    rc = lib().shapley_server_wait(srv, C.c_uint64(ticket), int(max_steps), C.byref(st))
    if rc == SHAPLEY_EAGAIN:
        return None
    _check(rc, (SHAPLEY_OK, SHAPLEY_ENOCONV))
    d = st.as_dict()
    d["rc"] = rc
    return d


def shapley_server_info(srv) -> dict:
    st = shapley_server_stats()
    _check(lib().shapley_server_info(srv, C.byref(st)))
    return {f: getattr(st, f) for f, _ in st._fields_ if f != "reserved"}


def shapley_server_destroy(srv) -> None:
    lib().shapley_server_destroy(srv)


def shapley_probe_enable(family, on: bool = True) -> None:
    fam = PROBE[family] if isinstance(family, str) else int(family)
    _check(lib().shapley_probe_enable(fam, 1 if on else 0))


def shapley_probe_read(family) -> dict:
    fam = PROBE[family] if isinstance(family, str) else int(family)
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().shapley_probe_read(fam, C.byref(n), C.byref(ms), C.byref(b)))
    return dict(launches=n.value, ms=ms.value, bytes=b.value)


def shapley_tune_lanes(lanes: int = 0) -> None:
    """Lanes per sparse row in the cycle kernels: 0 tunes per level, 1/2/4 force."""
    _check(lib().shapley_tune_lanes(int(lanes)))


def shapley_tune_galerkin(kernel: int = -1) -> None:
    """Galerkin product kernels: -1 chooses per product, 0 wavefront only, 1 thread per row first, 4 four lanes
    per row first."""
    _check(lib().shapley_tune_galerkin(int(kernel)))


def shapley_debug_fail_alloc(after: int) -> None:
    """Testing aid: the after-th device allocation from now fails with ENOMEM (0 disarms)."""
    _check(lib().shapley_debug_fail_alloc(int(after)))


def shapley_tune_interp(kernel: int = -1) -> None:
    """Coarse-level interpolation kernels: -1 four lanes per row first on large levels, 4 on every level,
    0 wavefront only."""
    _check(lib().shapley_tune_interp(int(kernel)))


def shapley_tune_dense(kernel: int = -1) -> None:
    """Coarsest-level inverse of blocks up to 64 unknowns: -1 FP64 matrix-core sweep, 0 register Gauss-Jordan."""
    _check(lib().shapley_tune_dense(int(kernel)))


def shapley_coarse_inverse(blocks) -> list:
    """Inverses of dense square blocks (a list of 2-D arrays) computed by the coarsest-level kernels."""
    mats = [np.ascontiguousarray(b, dtype=np.float64) for b in blocks]
    for m in mats:
        if m.ndim != 2 or m.shape[0] != m.shape[1]:
            raise ValueError("blocks must be square matrices")
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    flat = np.concatenate([m.ravel() for m in mats]) if mats else np.zeros(0)
    out = np.empty_like(flat)
    _check(lib().shapley_coarse_inverse(_ptr(flat), _ptr(sizes), int(len(mats)), _ptr(out)))
    res, off = [], 0
    for m in mats:
        k = m.size
        res.append(out[off:off + k].reshape(m.shape))
        off += k
    return res


def shapley_tune_stencil(mode: int = -1) -> None:
    """Compact matrix forms of the cycle (stencil finest level, 16-bit column offsets): -1 where they apply,
    0 CSR with 32-bit columns only."""
    _check(lib().shapley_tune_stencil(int(mode)))


def shapley_probe_read_large(family, frac: float = 0.5) -> dict:
    fam = PROBE[family] if isinstance(family, str) else int(family)
    n, ms, b = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().shapley_probe_read_large(fam, float(frac), C.byref(n), C.byref(ms), C.byref(b)))
    return dict(launches=n.value, ms=ms.value, bytes=b.value)


# ---------------------------------------------------------------------------
# convenience: a game object with the attributes n, m1, m2, row_ptr, col, w,
# r, mu, valid and optionally grid (dim, s, bvals)
# ---------------------------------------------------------------------------

def create_from(game, stream=None, device=False):
    """Handle of a game object; device=True first copies its arrays into torch
    device tensors and creates from their pointers (SHAPLEY_DEVICE_PTRS)."""
    grid = None
    gr = getattr(game, "grid", None)
    if gr is not None and not getattr(gr, "periodic", False):
        grid = (gr.dim, gr.s, gr.bvals)
    if not device:
        return shapley_game_create(game.n, game.m1, game.m2, game.row_ptr, game.col, game.w, game.r,
                                   game.mu, getattr(game, "valid", None), grid, 0, stream)
    import torch

    def t(a, dt):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()

    if grid is not None:
        grid = (grid[0], grid[1], t(grid[2], np.float64))
    args = (t(game.row_ptr, np.int64), t(game.col, np.int32), t(game.w, np.float64), t(game.r, np.float64))
    valid = t(getattr(game, "valid", None), np.uint8)
    torch.cuda.synchronize()  # the copies are complete before the library reads them
    return shapley_game_create(game.n, game.m1, game.m2, *args, game.mu, valid, grid, SHAPLEY_DEVICE_PTRS,
                               stream)
