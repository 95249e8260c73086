"""Python binding of the C ABI in ``include/ct.h`` (argument marshalling only).

Functions keep the C names.  Device arrays are torch tensors on the current
HIP device (float32, contiguous); streams default to torch's current stream.
Every projection, step and reduction runs in the HIP library: if
``libctcsgd.so`` is missing this module raises on import of the library,
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctcsgd.so")

CT_OK, CT_NOT_CONVERGED = 0, 1
CT_EINVAL, CT_ENOMEM, CT_EDEVICE, CT_EUNSUPPORTED = -1, -2, -3, -4
CT_ACCUMULATE = 1
CT_SAMPLE_DENSITY, CT_SAMPLE_UNIFORM, CT_SAMPLE_MIXED = 0, 1, 2
CT_SYNC_COLUMN, CT_SYNC_EPOCH = 0, 1
CT_BATCH_GRAPH = 1
CT_TUNE_REFRESH = 1

EXPORTS = (
    "ct_geom_create", "ct_geom_destroy", "ct_geom_get_info", "ct_geom_block_nnz",
    "ct_geom_block_nnz_static",
    "ct_geom_block_area", "ct_schedule_create_w",
    "ct_block_fwd", "ct_block_back",
    "ct_schedule_create", "ct_schedule_import", "ct_schedule_export", "ct_schedule_destroy",
    "ct_solver_workspace_bytes", "ct_solver_create", "ct_solver_destroy", "ct_solver_reset",
    "ct_block_epoch", "ct_solver_state", "ct_true_residual", "ct_residual_norms", "ct_solve",
    "ct_solver_profile", "ct_solver_profile_read",
    "ct_batch_create", "ct_batch_destroy", "ct_batch_add", "ct_batch_remove", "ct_batch_epoch",
    "ct_batch_job_epoch", "ct_batch_profile", "ct_batch_profile_read",
    "ct_geom_set_tuning", "ct_geom_get_tuning", "ct_geom_tune", "ct_batch_tune", "ct_batch_set_tuning",
    "ct_server_create", "ct_server_destroy", "ct_server_submit", "ct_server_tick", "ct_server_poll",
    "ct_server_result", "ct_job_footprint",
    "ct_last_error",
)


class CtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ct error {code}: {msg}")
        self.code = code


P = ctypes.c_void_p
i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64


class ct_geom_desc(ctypes.Structure):
    _fields_ = [("kind", i32), ("nx", i32), ("ny", i32), ("nz", i32),
                ("vx", f64), ("vy", f64), ("vz", f64), ("ox", f64), ("oy", f64), ("oz", f64),
                ("n_views", i32), ("nu", i32), ("nv", i32), ("pu", f64), ("pv", f64),
                ("views", P), ("n_row_blocks", i32), ("rb_ptr", P), ("tiles", P),
                ("n_col_blocks", i32), ("boxes", P)]


class ct_geom_info(ctypes.Structure):
    _fields_ = [("n_rays", i64), ("n_vox", i64), ("m", i32), ("n", i32),
                ("max_rb_rays", i32), ("max_cb_vox", i32)]


class ct_sched_params(ctypes.Structure):
    _fields_ = [("epochs", i32), ("alpha", f64), ("gamma", f64), ("group_size", i32),
                ("b", f64), ("sampling", i32), ("theta_step", f64), ("seed", u64)]


class ct_sched_view(ctypes.Structure):
    _fields_ = [("n_epochs", i32), ("n_cols", i32), ("n_groups", i32), ("n_rbs", i32),
                ("epoch_col_ptr", P), ("cols", P), ("col_group_ptr", P),
                ("group_rb_ptr", P), ("rbs", P), ("beta", P)]


class ct_kernel_times(ctypes.Structure):
    _fields_ = [("ms", f64 * 8), ("launches", i64 * 8)]


KERNEL_NAMES = ("back", "fwd", "step", "finalize", "residual")


class ct_batch_job(ctypes.Structure):
    _fields_ = [("solver", P), ("sched", P), ("y", P), ("x", P), ("epoch", i32)]


class ct_solver_params(ctypes.Structure):
    _fields_ = [("sync", i32)]


class ct_server_params(ctypes.Structure):
    _fields_ = [("capacity", i32), ("hbm_budget", i64), ("rel_tol", f64), ("check_every", i32),
                ("tau", f64), ("use_graph", i32)]


class ct_server_job(ctypes.Structure):
    _fields_ = [("geom", ctypes.POINTER(ct_geom_desc)), ("sched", ct_sched_params),
                ("solver", ct_solver_params), ("y", P), ("tag", i64)]


class ct_server_done(ctypes.Structure):
    _fields_ = [("tag", i64), ("id", i32), ("status", i32), ("epochs", i32), ("rel_residual", f64),
                ("t_submit", f64), ("t_admit", f64), ("t_done", f64), ("bytes", i64),
                ("updates", i64)]


class ct_server_stats(ctypes.Structure):
    _fields_ = [("active", i32), ("queued", i32), ("admitted", i64), ("retired", i64),
                ("updates", i64), ("bytes_in_use", i64), ("budget", i64), ("now", f64)]


class ct_tuning(ctypes.Structure):
    _fields_ = [("fwd_split", i32), ("back_waves", i32), ("ms", f64), ("ms_default", f64),
                ("trials", i32), ("cached", i32)]


class ct_solve_params(ctypes.Structure):
    _fields_ = [("sched", ct_sched_params), ("solver", ct_solver_params), ("tau", f64),
                ("rel_tol", f64), ("check_every", i32)]


class ct_solve_stats(ctypes.Structure):
    _fields_ = [("epochs_run", i32), ("rel_residual", f64), ("ray_voxel_updates", i64),
                ("r_norm", P)]


_lib = None


def lib():
    """Load ``libctcsgd.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_1709_00953_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "ct_geom_create": [ctypes.POINTER(ct_geom_desc), ctypes.POINTER(P)],
            "ct_geom_destroy": [P],
            "ct_geom_get_info": [P, ctypes.POINTER(ct_geom_info)],
            "ct_geom_block_nnz": [P, f64, P, P],
            "ct_geom_block_nnz_static": [P, f64, P, P],
            "ct_geom_block_area": [P, P],
            "ct_schedule_create_w": [P, ctypes.POINTER(ct_sched_params), P, ctypes.POINTER(P)],
            "ct_block_fwd": [P, P, i32, i32, P, P, i32, P],
            "ct_block_back": [P, P, i32, i32, P, P, i32, P],
            "ct_schedule_create": [P, ctypes.POINTER(ct_sched_params), P, ctypes.POINTER(P)],
            "ct_schedule_import": [P, ctypes.POINTER(ct_sched_view), ctypes.POINTER(P)],
            "ct_schedule_export": [P, ctypes.POINTER(ct_sched_view)],
            "ct_schedule_destroy": [P],
            "ct_solver_workspace_bytes": [P, ctypes.POINTER(ct_solver_params),
                                          ctypes.POINTER(ctypes.c_size_t)],
            "ct_solver_create": [P, ctypes.POINTER(ct_solver_params), P, ctypes.c_size_t,
                                 ctypes.POINTER(P)],
            "ct_solver_destroy": [P],
            "ct_solver_reset": [P, P, P, P],
            "ct_block_epoch": [P, P, i32, P, P, P],
            "ct_solver_state": [P, ctypes.POINTER(P), ctypes.POINTER(P)],
            "ct_true_residual": [P, P, P, ctypes.POINTER(f64), P],
            "ct_residual_norms": [P, P, P, P, P],
            "ct_server_create": [ctypes.POINTER(ct_server_params), ctypes.POINTER(P)],
            "ct_server_destroy": [P],
            "ct_server_submit": [P, ctypes.POINTER(ct_server_job), ctypes.POINTER(i32)],
            "ct_server_tick": [P, P, ctypes.POINTER(ct_server_stats)],
            "ct_server_poll": [P, ctypes.POINTER(ct_server_done), i32, ctypes.POINTER(i32)],
            "ct_server_result": [P, i32, P],
            "ct_solve": [P, ctypes.POINTER(ct_solve_params), P, P, P, ctypes.c_size_t,
                         ctypes.POINTER(ct_solve_stats), P],
            "ct_solver_profile": [P, i32],
            "ct_solver_profile_read": [P, ctypes.POINTER(ct_kernel_times)],
            "ct_batch_create": [i32, ctypes.POINTER(P)],
            "ct_batch_destroy": [P],
            "ct_batch_add": [P, ctypes.POINTER(ct_batch_job), ctypes.POINTER(i32)],
            "ct_batch_remove": [P, i32],
            "ct_batch_epoch": [P, i32, ctypes.POINTER(i32), P],
            "ct_batch_job_epoch": [P, i32, ctypes.POINTER(i32)],
            "ct_batch_profile": [P, i32],
            "ct_batch_profile_read": [P, ctypes.POINTER(ct_kernel_times)],
            "ct_geom_set_tuning": [P, ctypes.POINTER(ct_tuning)],
            "ct_geom_get_tuning": [P, ctypes.POINTER(ct_tuning)],
            "ct_geom_tune": [P, P, i32, ctypes.POINTER(ct_tuning), P],
            "ct_batch_tune": [P, i32, P, P],
            "ct_batch_set_tuning": [P, i32, ctypes.POINTER(ct_tuning)],
            "ct_job_footprint": [ctypes.POINTER(ct_geom_desc), ctypes.POINTER(ct_solver_params),
                                 ctypes.POINTER(ctypes.c_size_t)],
            "ct_last_error": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name.endswith("_destroy") else ctypes.c_int
        L.ct_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def ct_last_error() -> str:
    return lib().ct_last_error().decode()


def _check(rc: int, allow=(CT_OK,)) -> int:
    if rc not in allow:
        raise CtError(rc, ct_last_error())
    return rc


def _stream(stream):
    if stream is not None:
        return P(stream)
    import torch
    return P(torch.cuda.current_stream().cuda_stream)


def _dev(t, n: Optional[int] = None, name: str = "array"):
    """Pointer of a contiguous float32 device tensor with n elements."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float32")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return P(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(P)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
class Geom:
    """Owns a ``ct_geom*`` and the host arrays its description referenced."""

    def __init__(self, handle, g):
        self.handle = handle
        self.g = g
        info = ct_geom_info()
        _check(lib().ct_geom_get_info(handle, ctypes.byref(info)))
        self.M, self.N = int(info.n_rays), int(info.n_vox)
        self.m, self.n = int(info.m), int(info.n)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.ct_geom_destroy(h)


def make_desc(g):
    """Marshal an ``inputs.Geometry`` into a ``ct_geom_desc`` (+ keep-alive list)."""
    views = np.ascontiguousarray(g.views, dtype=np.float64)
    rb_ptr = np.zeros(len(g.row_blocks) + 1, dtype=np.int32)
    rb_ptr[1:] = np.cumsum([len(b) for b in g.row_blocks])
    tiles = np.ascontiguousarray(np.concatenate(g.row_blocks, axis=0), dtype=np.int32)
    boxes = np.ascontiguousarray(g.col_blocks, dtype=np.int32)
    d = ct_geom_desc(g.kind, g.nx, g.ny, g.nz, g.vx, g.vy, g.vz, g.ox, g.oy, g.oz,
                     g.n_views, g.nu, g.nv, g.pu, g.pv, _np_ptr(views), len(g.row_blocks),
                     _np_ptr(rb_ptr), _np_ptr(tiles), len(boxes), _np_ptr(boxes))
    return d, (views, rb_ptr, tiles, boxes)


def ct_geom_create(g) -> Geom:
    d, keep = make_desc(g)
    h = P()
    _check(lib().ct_geom_create(ctypes.byref(d), ctypes.byref(h)))
    return Geom(h, g)


def ct_geom_block_nnz(geom: Geom, tau: float, stream=None) -> np.ndarray:
    out = np.zeros((geom.m, geom.n), dtype=np.int64)
    _check(lib().ct_geom_block_nnz(geom.handle, float(tau), _np_ptr(out), _stream(stream)))
    return out


def ct_geom_block_nnz_static(geom: Geom, tau: float, out: np.ndarray | None = None,
                             stream=None) -> np.ndarray:
    """ct_geom_block_nnz with the library's static counter array (no
    allocation by the library; ``out``, an int64 [m, n] host array, may be
    passed in so that the call allocates nothing here either)."""
    if out is None:
        out = np.zeros((geom.m, geom.n), dtype=np.int64)
    if out.dtype != np.int64 or out.shape != (geom.m, geom.n) or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous int64 array of shape (m, n)")
    _check(lib().ct_geom_block_nnz_static(geom.handle, float(tau), _np_ptr(out), _stream(stream)))
    return out


def ct_geom_block_area(geom: Geom) -> np.ndarray:
    """P_S per (row block, column block), float64 [m, n] (host only)."""
    out = np.zeros((geom.m, geom.n), dtype=np.float64)
    _check(lib().ct_geom_block_area(geom.handle, _np_ptr(out)))
    return out


def ct_job_footprint(g, sync: int = CT_SYNC_COLUMN) -> int:
    d, keep = make_desc(g)
    sp = ct_solver_params(sync)
    n = ctypes.c_size_t()
    _check(lib().ct_job_footprint(ctypes.byref(d), ctypes.byref(sp), ctypes.byref(n)))
    return int(n.value)


# ----------------------------------------------------------------------------
# primitives
# ----------------------------------------------------------------------------
def _rbs(row_blocks: Sequence[int]):
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(row_blocks, dtype=np.int32)))
    return a, len(a)


def ct_block_fwd(geom: Geom, row_blocks, col_block: int, x, y, flags: int = 0, stream=None):
    rb, n = _rbs(row_blocks)
    _check(lib().ct_block_fwd(geom.handle, _np_ptr(rb), n, int(col_block), _dev(x, geom.N, "x"),
                              _dev(y, geom.M, "y"), int(flags), _stream(stream)))


def ct_block_back(geom: Geom, row_blocks, col_block: int, r, g, flags: int = 0, stream=None):
    rb, n = _rbs(row_blocks)
    _check(lib().ct_block_back(geom.handle, _np_ptr(rb), n, int(col_block), _dev(r, geom.M, "r"),
                               _dev(g, geom.N, "g"), int(flags), _stream(stream)))


# ----------------------------------------------------------------------------
# schedules
# ----------------------------------------------------------------------------
class Schedule:
    def __init__(self, handle, geom):
        self.handle = handle
        self.geom = geom        # keeps the geometry alive

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.ct_schedule_destroy(h)


def sched_params(epochs, alpha=1.0, gamma=1.0, group_size=1, b=1.0,
                 sampling=CT_SAMPLE_DENSITY, theta_step=0.0, seed=0) -> ct_sched_params:
    return ct_sched_params(int(epochs), float(alpha), float(gamma), int(group_size), float(b),
                           int(sampling), float(theta_step), int(seed) & ((1 << 64) - 1))


def ct_schedule_create(geom: Geom, params: ct_sched_params, nnz) -> Schedule:
    nnz = np.ascontiguousarray(nnz, dtype=np.int64)
    if nnz.shape != (geom.m, geom.n):
        raise ValueError(f"nnz must be {(geom.m, geom.n)}")
    h = P()
    _check(lib().ct_schedule_create(geom.handle, ctypes.byref(params), _np_ptr(nnz), ctypes.byref(h)))
    return Schedule(h, geom)


def ct_schedule_create_w(geom: Geom, params: ct_sched_params, w) -> Schedule:
    """Schedule from any nonnegative block density weights [m, n]."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    if w.shape != (geom.m, geom.n):
        raise ValueError(f"weights must be [{geom.m}, {geom.n}]")
    h = P()
    _check(lib().ct_schedule_create_w(geom.handle, ctypes.byref(params), _np_ptr(w), ctypes.byref(h)))
    return Schedule(h, geom)


def ct_schedule_import(geom: Geom, s) -> Schedule:
    """``s`` has the flat arrays epoch_col_ptr, cols, col_group_ptr,
    group_rb_ptr, rbs, beta (e.g. an oracle schedule)."""
    arrs = [np.ascontiguousarray(getattr(s, k), dtype=np.int32)
            for k in ("epoch_col_ptr", "cols", "col_group_ptr", "group_rb_ptr", "rbs")]
    beta = np.ascontiguousarray(s.beta, dtype=np.float64)
    v = ct_sched_view(len(arrs[0]) - 1, len(arrs[1]), len(beta), len(arrs[4]),
                      *[_np_ptr(a) for a in arrs], _np_ptr(beta))
    h = P()
    _check(lib().ct_schedule_import(geom.handle, ctypes.byref(v), ctypes.byref(h)))
    return Schedule(h, geom)


def ct_schedule_export(sched: Schedule) -> dict:
    v = ct_sched_view()
    _check(lib().ct_schedule_export(sched.handle, ctypes.byref(v)))

    def arr(ptr, n, ct, dt):
        if n == 0:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(n,)).astype(dt)

    E, C, G, R = v.n_epochs, v.n_cols, v.n_groups, v.n_rbs
    return {"epoch_col_ptr": arr(v.epoch_col_ptr, E + 1, ctypes.c_int32, np.int32),
            "cols": arr(v.cols, C, ctypes.c_int32, np.int32),
            "col_group_ptr": arr(v.col_group_ptr, C + 1, ctypes.c_int32, np.int32),
            "group_rb_ptr": arr(v.group_rb_ptr, G + 1, ctypes.c_int32, np.int32),
            "rbs": arr(v.rbs, R, ctypes.c_int32, np.int32),
            "beta": arr(v.beta, G, ctypes.c_double, np.float64)}


# ----------------------------------------------------------------------------
# solver
# ----------------------------------------------------------------------------
class Solver:
    def __init__(self, handle, geom, ws, sync):
        self.handle = handle
        self.geom = geom
        self.ws = ws            # torch uint8 workspace (caller-owned device memory)
        self.sync = sync

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.ct_solver_destroy(h)


def ct_solver_workspace_bytes(geom: Geom, sync: int = CT_SYNC_COLUMN) -> int:
    sp = ct_solver_params(sync)
    n = ctypes.c_size_t()
    _check(lib().ct_solver_workspace_bytes(geom.handle, ctypes.byref(sp), ctypes.byref(n)))
    return int(n.value)


def ct_solver_create(geom: Geom, sync: int = CT_SYNC_COLUMN, workspace=None) -> Solver:
    import torch
    nbytes = ct_solver_workspace_bytes(geom, sync)
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = workspace.data_ptr()
    off = (-base) % 256
    sp = ct_solver_params(sync)
    h = P()
    _check(lib().ct_solver_create(geom.handle, ctypes.byref(sp), P(base + off),
                                  workspace.numel() - off, ctypes.byref(h)))
    return Solver(h, geom, workspace, sync)


def ct_solver_reset(solver: Solver, y, x=None, stream=None):
    g = solver.geom
    xp = _dev(x, g.N, "x") if x is not None else P()
    _check(lib().ct_solver_reset(solver.handle, _dev(y, g.M, "y"), xp, _stream(stream)))


def ct_block_epoch(solver: Solver, sched: Schedule, epoch: int, y, x, stream=None):
    g = solver.geom
    _check(lib().ct_block_epoch(solver.handle, sched.handle, int(epoch), _dev(y, g.M, "y"),
                                _dev(x, g.N, "x"), _stream(stream)))


def ct_solver_state(solver: Solver):
    """(z [n, M], r [M]) as torch views into the solver workspace."""
    import torch
    zp, rp = P(), P()
    _check(lib().ct_solver_state(solver.handle, ctypes.byref(zp), ctypes.byref(rp)))
    g = solver.geom
    base = solver.ws.data_ptr()
    ws = solver.ws

    def view(ptr, n):
        off = ptr - base
        return ws[off:off + 4 * n].view(torch.float32)

    return view(zp.value, g.n * g.M).view(g.n, g.M), view(rp.value, g.M)


def ct_true_residual(solver: Solver, y, x, stream=None) -> float:
    g = solver.geom
    rel = f64()
    _check(lib().ct_true_residual(solver.handle, _dev(y, g.M, "y"), _dev(x, g.N, "x"),
                                  ctypes.byref(rel), _stream(stream)))
    return float(rel.value)


def ct_residual_norms(solver: Solver, y, x, out, stream=None):
    """Asynchronous: out (device float64 [2]) <- ||y - A x||^2, ||y||^2."""
    import torch
    g = solver.geom
    if out.dtype != torch.float64 or out.numel() < 2 or not out.is_cuda:
        raise ValueError("out must be a device float64 tensor of 2 elements")
    _check(lib().ct_residual_norms(solver.handle, _dev(y, g.M, "y"), _dev(x, g.N, "x"),
                                   P(out.data_ptr()), _stream(stream)))


def ct_solver_profile(solver: Solver, enable: bool = True):
    _check(lib().ct_solver_profile(solver.handle, 1 if enable else 0))


def ct_solver_profile_read(solver: Solver) -> dict:
    """{kernel: (ms, launches)} since the last read (synchronises)."""
    t = ct_kernel_times()
    _check(lib().ct_solver_profile_read(solver.handle, ctypes.byref(t)))
    return {name: (float(t.ms[k]), int(t.launches[k])) for k, name in enumerate(KERNEL_NAMES)}


def ct_solve(geom: Geom, params: ct_sched_params, y, x, sync=CT_SYNC_COLUMN, tau=0.0,
             rel_tol=0.0, check_every=0, workspace=None, stream=None):
    """Whole solve; the workspace is a caller tensor (allocated here if not
    given).  Returns (status, stats) with the per-epoch ||r|| in stats."""
    import torch
    sp = ct_solve_params(params, ct_solver_params(sync), float(tau), float(rel_tol), int(check_every))
    nbytes = ct_solver_workspace_bytes(geom, sync)
    if workspace is None:
        workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = workspace.data_ptr()
    off = (-base) % 256
    rn = np.zeros(max(1, params.epochs), dtype=np.float64)
    st = ct_solve_stats()
    st.r_norm = rn.ctypes.data_as(P)
    rc = _check(lib().ct_solve(geom.handle, ctypes.byref(sp), _dev(y, geom.M, "y"),
                               _dev(x, geom.N, "x"), P(base + off), workspace.numel() - off,
                               ctypes.byref(st), _stream(stream)),
                allow=(CT_OK, CT_NOT_CONVERGED))
    return rc, {"epochs_run": st.epochs_run, "rel_residual": st.rel_residual,
                "ray_voxel_updates": st.ray_voxel_updates,
                "r_norm": rn[:st.epochs_run].copy()}


# ----------------------------------------------------------------------------
# batch
# ----------------------------------------------------------------------------
class Batch:
    """A batch handle; keeps the Python objects of its jobs alive while they
    are members."""

    def __init__(self, handle):
        self.handle = handle
        self.members = {}       # id -> (solver, sched, y, x)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.ct_batch_destroy(h)


def ct_batch_create(capacity: int) -> Batch:
    h = P()
    _check(lib().ct_batch_create(int(capacity), ctypes.byref(h)))
    return Batch(h)


def ct_batch_add(batch: Batch, solver: Solver, sched: Schedule, y, x, epoch: int = 0) -> int:
    g = solver.geom
    job = ct_batch_job(solver.handle, sched.handle, _dev(y, g.M, "y"), _dev(x, g.N, "x"), int(epoch))
    jid = i32()
    _check(lib().ct_batch_add(batch.handle, ctypes.byref(job), ctypes.byref(jid)))
    batch.members[int(jid.value)] = (solver, sched, y, x)
    return int(jid.value)


def ct_batch_remove(batch: Batch, jid: int):
    _check(lib().ct_batch_remove(batch.handle, int(jid)))
    batch.members.pop(int(jid), None)


def ct_batch_epoch(batch: Batch, graph: bool = False, stream=None) -> int:
    """One batch epoch; returns the number of jobs that had an epoch to run."""
    ran = i32()
    _check(lib().ct_batch_epoch(batch.handle, CT_BATCH_GRAPH if graph else 0, ctypes.byref(ran),
                                _stream(stream)))
    return int(ran.value)


def ct_batch_job_epoch(batch: Batch, jid: int) -> int:
    e = i32()
    _check(lib().ct_batch_job_epoch(batch.handle, int(jid), ctypes.byref(e)))
    return int(e.value)


def ct_batch_profile(batch: Batch, enable: bool = True):
    _check(lib().ct_batch_profile(batch.handle, 1 if enable else 0))


def ct_batch_profile_read(batch: Batch) -> dict:
    """{kernel: (ms, launches)} of the batched launches since the last read."""
    t = ct_kernel_times()
    _check(lib().ct_batch_profile_read(batch.handle, ctypes.byref(t)))
    return {name: (float(t.ms[k]), int(t.launches[k])) for k, name in enumerate(KERNEL_NAMES)}


# ----------------------------------------------------------------------------
# launch shapes and their tuner
# ----------------------------------------------------------------------------
def _tuning_dict(t: ct_tuning) -> dict:
    return {"fwd_split": int(t.fwd_split), "back_waves": int(t.back_waves), "ms": float(t.ms),
            "ms_default": float(t.ms_default), "trials": int(t.trials), "cached": bool(t.cached)}


def ct_geom_set_tuning(geom: Geom, fwd_split: int, back_waves: int):
    t = ct_tuning(int(fwd_split), int(back_waves), 0.0, 0.0, 0, 0)
    _check(lib().ct_geom_set_tuning(geom.handle, ctypes.byref(t)))


def ct_geom_get_tuning(geom: Geom) -> dict:
    t = ct_tuning()
    _check(lib().ct_geom_get_tuning(geom.handle, ctypes.byref(t)))
    return _tuning_dict(t)


def ct_geom_tune(geom: Geom, sched: Schedule, refresh: bool = False, stream=None) -> dict:
    t = ct_tuning()
    _check(lib().ct_geom_tune(geom.handle, sched.handle, CT_TUNE_REFRESH if refresh else 0,
                              ctypes.byref(t), _stream(stream)))
    return _tuning_dict(t)


def ct_batch_tune(batch: Batch, refresh: bool = False, stream=None) -> list:
    """Per geometry kind (index = kind), the chosen shapes (None for kinds no
    job has)."""
    out = (ct_tuning * 4)()
    _check(lib().ct_batch_tune(batch.handle, CT_TUNE_REFRESH if refresh else 0, out, _stream(stream)))
    return [(_tuning_dict(out[k]) if out[k].fwd_split else None) for k in range(4)]


def ct_batch_set_tuning(batch: Batch, kind: int, fwd_split: int, back_waves: int):
    t = ct_tuning(int(fwd_split), int(back_waves), 0.0, 0.0, 0, 0)
    _check(lib().ct_batch_set_tuning(batch.handle, int(kind), ctypes.byref(t)))


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
class Server:
    def __init__(self, handle):
        self.handle = handle
        self.n_vox = {}         # job id -> N

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.ct_server_destroy(h)


def ct_server_create(capacity=16, hbm_budget=0, rel_tol=1e-3, check_every=10, tau=0.0,
                     graph=True) -> Server:
    p = ct_server_params(int(capacity), int(hbm_budget), float(rel_tol), int(check_every), float(tau),
                         1 if graph else 0)
    h = P()
    _check(lib().ct_server_create(ctypes.byref(p), ctypes.byref(h)))
    return Server(h)


def ct_server_submit(server: Server, g, params: ct_sched_params, y, sync=CT_SYNC_COLUMN, tag=0) -> int:
    """Queue a job: geometry ``g`` (inputs.Geometry), schedule parameters,
    host measurements ``y`` (float32 [M])."""
    d, keep = make_desc(g)
    yh = np.ascontiguousarray(y, dtype=np.float32)
    if yh.size != g.n_rays:
        raise ValueError(f"y has {yh.size} values, the geometry {g.n_rays} rays")
    job = ct_server_job(ctypes.pointer(d), params, ct_solver_params(sync), _np_ptr(yh), int(tag))
    jid = i32()
    _check(lib().ct_server_submit(server.handle, ctypes.byref(job), ctypes.byref(jid)))
    server.n_vox[int(jid.value)] = g.n_vox
    return int(jid.value)


def ct_server_tick(server: Server, stream=None) -> dict:
    st = ct_server_stats()
    _check(lib().ct_server_tick(server.handle, _stream(stream), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in ct_server_stats._fields_}


def ct_server_poll(server: Server, max_n: int = 256) -> list:
    arr = (ct_server_done * max_n)()
    n = i32()
    _check(lib().ct_server_poll(server.handle, arr, int(max_n), ctypes.byref(n)))
    return [{k: getattr(arr[i], k) for k, _ in ct_server_done._fields_} for i in range(n.value)]


def ct_server_result(server: Server, jid: int) -> np.ndarray:
    if int(jid) not in server.n_vox:
        raise CtError(CT_EINVAL, f"no job {jid} was submitted to this server")
    x = np.zeros(server.n_vox[int(jid)], dtype=np.float32)
    _check(lib().ct_server_result(server.handle, int(jid), _np_ptr(x)))
    return x
