"""Thin ctypes binding of the C ABI in include/wbpr.h (argument marshalling only).

Every step of the solve runs in the HIP library ``libwbpr.so``; this module
only converts Python/numpy/torch arguments to pointers.  If the library is
missing it raises instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwbpr.so")

WBPR_OK = 0
WBPR_EINVAL = 1
WBPR_ENOMEM = 2
WBPR_ETOOBIG = 3
WBPR_ETIMEOUT = 4
WBPR_EDEVICE = 5
WBPR_EAGAIN = 6
WBPR_EOVERFLOW = 7
WBPR_EINTERNAL = 8
WBPR_ECANCELED = 9

STATUS_NAMES = {
    0: "WBPR_OK", 1: "WBPR_EINVAL", 2: "WBPR_ENOMEM", 3: "WBPR_ETOOBIG", 4: "WBPR_ETIMEOUT",
    5: "WBPR_EDEVICE", 6: "WBPR_EAGAIN", 7: "WBPR_EOVERFLOW", 8: "WBPR_EINTERNAL", 9: "WBPR_ECANCELED",
}

# Every symbol declared in include/wbpr.h.
EXPORTS = (
    "wbpr_version", "wbpr_last_error", "wbpr_device_arch", "wbpr_ctx_create", "wbpr_ctx_destroy",
    "wbpr_ctx_set_options", "wbpr_solve", "wbpr_solve_device", "wbpr_solve_batch", "wbpr_solve_batch_device",
    "wbpr_graph_upload", "wbpr_graph_solve", "wbpr_graph_free", "wbpr_autotune", "wbpr_wave_trace",
    "wbpr_bfs_farthest", "wbpr_pick_terminals", "wbpr_solve_multi",
    "wbpr_server_create", "wbpr_server_submit", "wbpr_server_poll", "wbpr_server_wait", "wbpr_result_free",
    "wbpr_server_get_stats", "wbpr_server_footprint", "wbpr_server_destroy", "wbpr_solve_device_noalloc",
)


class wbpr_csr(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int32),
        ("E", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("cap", ctypes.c_void_p),
    ]


class wbpr_options(ctypes.Structure):
    _fields_ = [
        ("layout", ctypes.c_int32),
        ("lanes_per_vertex", ctypes.c_int32),
        ("split_degree", ctypes.c_int32),
        ("gr_every_sweeps", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int64),
        ("max_wall_ms", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("time_kernels", ctypes.c_int32),
        ("push_mode", ctypes.c_int32),
        ("block_degree", ctypes.c_int32),
        ("gr_work_permille", ctypes.c_int32),
        ("no_graph", ctypes.c_int32),
        ("avq_mode", ctypes.c_int32),
        ("gr_stagnation", ctypes.c_int32),
        ("wave_trace", ctypes.c_int32),
        ("lds_max_v", ctypes.c_int32),
        ("gap", ctypes.c_int32),
        ("batch_kernel", ctypes.c_int32),
        ("debug_checks", ctypes.c_int32),
    ]


class wbpr_stats(ctypes.Structure):
    _fields_ = [
        ("value", ctypes.c_int64),
        ("V", ctypes.c_int64),
        ("E", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("sweeps", ctypes.c_int64),
        ("global_relabels", ctypes.c_int64),
        ("pushes", ctypes.c_int64),
        ("relabels", ctypes.c_int64),
        ("arc_scans", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("bfs_scans", ctypes.c_int64),
        ("phase2_sweeps", ctypes.c_int64),
        ("nonempty_sweeps", ctypes.c_int64),
        ("gr_levels", ctypes.c_int64),
        ("lanes_per_vertex", ctypes.c_int32),
        ("split_degree", ctypes.c_int32),
        ("block_degree", ctypes.c_int32),
        ("gr_every_sweeps", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("gr_blocks", ctypes.c_int32),
        ("ms_build", ctypes.c_double),
        ("ms_phase1", ctypes.c_double),
        ("ms_phase2", ctypes.c_double),
        ("ms_decode", ctypes.c_double),
        ("ms_total", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * 4),
        ("kernel_launches", ctypes.c_int64 * 4),
        ("kernel_arc_scans", ctypes.c_int64 * 4),
        ("kernel_pushes", ctypes.c_int64 * 4),
        ("kernel_relabels", ctypes.c_int64 * 4),
        ("kernel_queued", ctypes.c_int64 * 4),
        ("bfs_topdown_scans", ctypes.c_int64),
        ("instances", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("lds_solved", ctypes.c_int64),
        ("lds_fallbacks", ctypes.c_int64),
        ("gap_skipped", ctypes.c_int64),
        ("kernel_build_ms", ctypes.c_double),
        ("layout", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("wg_solved", ctypes.c_int64),
        ("wg_fallbacks", ctypes.c_int64),
        ("debug_checked", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


class WbprError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

# Handles still open at interpreter exit are closed by an atexit hook, in
# dependency order (servers and uploaded graphs before the contexts they were
# made from), so no stream, arena, captured graph or worker thread of the
# library outlives Python's own shutdown and meets the HIP runtime's static
# teardown.
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_live_graphs: "weakref.WeakSet" = weakref.WeakSet()
_live_solvers: "weakref.WeakSet" = weakref.WeakSet()


def close_all() -> None:
    """Close every library handle this process still holds (idempotent)."""
    for live in (_live_servers, _live_graphs, _live_solvers):
        for h in list(live):
            try:
                h.close()
            except Exception:
                pass


atexit.register(close_all)


def _init_torch_first():
    """PyTorch-ROCm ships its own copy of the HIP runtime (libamdhip64.so,
    soname libamdhip64.so.7, the soname libwbpr.so asks for).  Loading torch
    first makes the dynamic loader resolve libwbpr.so's dependency to that
    already loaded copy, so the process holds one HIP runtime and torch's
    device pointers and streams are the library's too.  Loading libwbpr.so
    first would bring in the system copy as well."""
    try:
        import torch
    except Exception:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


class wbpr_server_options(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_int64),
        ("max_slots", ctypes.c_int32),
        ("arcs_per_vertex", ctypes.c_int32),
        ("want_flows", ctypes.c_int32),
        ("want_sides", ctypes.c_int32),
        ("max_admit", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 5),
    ]


class wbpr_result(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("V", ctypes.c_int32),
        ("E", ctypes.c_int64),
        ("value", ctypes.c_int64),
        ("arc_flow", ctypes.POINTER(ctypes.c_int32)),
        ("cut_side", ctypes.POINTER(ctypes.c_uint8)),
        ("latency_ms", ctypes.c_double),
        ("queue_ms", ctypes.c_double),
    ]


class wbpr_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "pending", "resident", "rounds",
                                               "admissions", "sweeps")] + \
        [(n, ctypes.c_double) for n in ("busy_ms", "solves_per_s", "p50_ms", "p99_ms", "max_ms")] + \
        [(n, ctypes.c_int64) for n in ("arena_bytes", "scratch_bytes", "staging_bytes", "output_bytes", "Vcap",
                                       "Mcap", "Ecap")] + \
        [("max_slots", ctypes.c_int32), ("peak_resident", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def load_library(path: str = LIB_PATH):
    """Load libwbpr.so and declare every entry point; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run __graft_entry__.build())")
    _init_torch_first()
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.wbpr_version.restype = ctypes.c_char_p
    lib.wbpr_version.argtypes = []
    lib.wbpr_last_error.restype = ctypes.c_char_p
    lib.wbpr_last_error.argtypes = []
    lib.wbpr_device_arch.restype = ctypes.c_int
    lib.wbpr_device_arch.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    lib.wbpr_ctx_create.restype = ctypes.c_int
    lib.wbpr_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(wbpr_options), ctypes.POINTER(vp)]
    lib.wbpr_ctx_destroy.restype = None
    lib.wbpr_ctx_destroy.argtypes = [vp]
    lib.wbpr_ctx_set_options.restype = ctypes.c_int
    lib.wbpr_ctx_set_options.argtypes = [vp, ctypes.POINTER(wbpr_options)]
    lib.wbpr_solve.restype = ctypes.c_int
    lib.wbpr_solve.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, i32, vp, vp, vp, ctypes.POINTER(wbpr_stats)]
    lib.wbpr_solve_device.restype = ctypes.c_int
    lib.wbpr_solve_device.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, i32, vp, vp, vp, vp,
                                      ctypes.POINTER(wbpr_stats)]
    lib.wbpr_solve_device_noalloc.restype = ctypes.c_int
    lib.wbpr_solve_device_noalloc.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, i32, vp, vp, vp, vp,
                                              ctypes.POINTER(wbpr_stats)]
    lib.wbpr_solve_batch.restype = ctypes.c_int
    lib.wbpr_solve_batch.argtypes = [vp, i32, ctypes.POINTER(wbpr_csr), vp, vp, vp, vp, vp,
                                     ctypes.POINTER(wbpr_stats), vp]
    lib.wbpr_solve_batch_device.restype = ctypes.c_int
    lib.wbpr_solve_batch_device.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                            ctypes.POINTER(wbpr_stats), vp]
    lib.wbpr_graph_upload.restype = ctypes.c_int
    lib.wbpr_graph_upload.argtypes = [vp, ctypes.POINTER(wbpr_csr), ctypes.POINTER(ctypes.c_void_p)]
    lib.wbpr_graph_solve.restype = ctypes.c_int
    lib.wbpr_graph_solve.argtypes = [vp, i32, i32, vp, vp, vp, ctypes.POINTER(wbpr_stats)]
    lib.wbpr_graph_free.restype = None
    lib.wbpr_graph_free.argtypes = [vp]
    lib.wbpr_autotune.restype = ctypes.c_int
    lib.wbpr_autotune.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, i32, i32, i32, ctypes.POINTER(wbpr_options),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.wbpr_bfs_farthest.restype = ctypes.c_int
    lib.wbpr_bfs_farthest.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, vp, vp, vp]
    lib.wbpr_pick_terminals.restype = ctypes.c_int
    lib.wbpr_pick_terminals.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, ctypes.c_uint64, vp, vp,
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.wbpr_solve_multi.restype = ctypes.c_int
    lib.wbpr_solve_multi.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, vp, vp, vp, vp, vp,
                                     ctypes.POINTER(wbpr_stats)]
    lib.wbpr_wave_trace.restype = ctypes.c_int
    lib.wbpr_wave_trace.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.wbpr_server_create.restype = ctypes.c_int
    lib.wbpr_server_create.argtypes = [vp, ctypes.POINTER(wbpr_server_options), ctypes.POINTER(ctypes.c_void_p)]
    lib.wbpr_server_submit.restype = ctypes.c_int
    lib.wbpr_server_submit.argtypes = [vp, ctypes.POINTER(wbpr_csr), i32, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.wbpr_server_poll.restype = ctypes.c_int
    lib.wbpr_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(wbpr_result)]
    lib.wbpr_server_wait.restype = ctypes.c_int
    lib.wbpr_server_wait.argtypes = [vp, ctypes.c_uint64, i32, ctypes.POINTER(wbpr_result)]
    lib.wbpr_result_free.restype = None
    lib.wbpr_result_free.argtypes = [ctypes.POINTER(wbpr_result)]
    lib.wbpr_server_get_stats.restype = ctypes.c_int
    lib.wbpr_server_get_stats.argtypes = [vp, ctypes.POINTER(wbpr_server_stats)]
    lib.wbpr_server_footprint.restype = ctypes.c_int
    lib.wbpr_server_footprint.argtypes = [i32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.wbpr_server_destroy.restype = None
    lib.wbpr_server_destroy.argtypes = [vp]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != WBPR_OK:
        raise WbprError(rc, wbpr_last_error())


def wbpr_version() -> str:
    return load_library().wbpr_version().decode()


def wbpr_last_error() -> str:
    return load_library().wbpr_last_error().decode(errors="replace")


def wbpr_device_arch(dev: int = 0) -> str:
    buf = ctypes.create_string_buffer(128)
    _check(load_library().wbpr_device_arch(dev, buf, 128))
    return buf.value.decode()


def make_options(**kw) -> wbpr_options:
    o = wbpr_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def wbpr_ctx_create(device: int = 0, **options) -> int:
    lib = load_library()
    h = ctypes.c_void_p()
    opt = make_options(**options) if options else None
    _check(lib.wbpr_ctx_create(device, ctypes.byref(opt) if opt is not None else None, ctypes.byref(h)))
    return h.value


def wbpr_ctx_destroy(ctx: int) -> None:
    load_library().wbpr_ctx_destroy(ctx)


def wbpr_ctx_set_options(ctx: int, **options) -> None:
    opt = make_options(**options)
    _check(load_library().wbpr_ctx_set_options(ctx, ctypes.byref(opt)))


@dataclass
class Result:
    value: int
    flow: np.ndarray | None
    side: np.ndarray | None
    stats: dict


def wbpr_solve(ctx: int, V: int, row_ptr, col, cap, s: int, t: int, want_flow: bool = True,
               want_side: bool = True, return_code: bool = False):
    """Solve from host arrays; returns Result (or the raw status when return_code)."""
    lib = load_library()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    k = np.ascontiguousarray(cap, dtype=np.int32)
    E = int(c.shape[0])
    g = wbpr_csr(V, E, rp.ctypes.data, c.ctypes.data if E else None, k.ctypes.data if E else None)
    value = ctypes.c_int64(0)
    flow = np.zeros(max(E, 1), np.int32) if want_flow else None
    side = np.zeros(max(V, 1), np.uint8) if want_side else None
    st = wbpr_stats()
    rc = lib.wbpr_solve(ctx, ctypes.byref(g), s, t, ctypes.addressof(value),
                        flow.ctypes.data if flow is not None else None,
                        side.ctypes.data if side is not None else None, ctypes.byref(st))
    if return_code:
        return rc
    _check(rc)
    return Result(int(value.value), flow[:E] if flow is not None else None,
                  side[:V] if side is not None else None, st.as_dict())


def _host_csr(g):
    """(wbpr_csr, arrays to keep alive) for a host graph object."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(g.col, dtype=np.int32)
    k = np.ascontiguousarray(g.cap, dtype=np.int32)
    E = int(c.shape[0])
    return wbpr_csr(g.V, E, rp.ctypes.data, c.ctypes.data if E else None, k.ctypes.data if E else None), (rp, c, k)


def wbpr_bfs_farthest(ctx: int, g, sources):
    """(eccentricity, farthest vertex) arrays for every vertex in sources."""
    lib = load_library()
    csr, keep = _host_csr(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    n = int(src.shape[0])
    ecc = np.zeros(max(n, 1), np.int32)
    far = np.zeros(max(n, 1), np.int32)
    _check(lib.wbpr_bfs_farthest(ctx, ctypes.byref(csr), n, src.ctypes.data if n else None,
                                 ecc.ctypes.data if n else None, far.ctypes.data if n else None))
    return ecc[:n], far[:n]


def wbpr_pick_terminals(ctx: int, g, k: int, seed: int):
    """(sources, sinks) chosen by the paper's BFS rule (at most k pairs)."""
    lib = load_library()
    csr, keep = _host_csr(g)
    src = np.zeros(max(k, 1), np.int32)
    snk = np.zeros(max(k, 1), np.int32)
    n = ctypes.c_int32(0)
    _check(lib.wbpr_pick_terminals(ctx, ctypes.byref(csr), k, seed, src.ctypes.data, snk.ctypes.data, ctypes.byref(n)))
    return src[: n.value], snk[: n.value]


def wbpr_solve_multi(ctx: int, g, sources, sinks, want_flow: bool = True, want_side: bool = True,
                     return_code: bool = False):
    """Multi-source, multi-sink maximum flow through a super-source and super-sink."""
    lib = load_library()
    csr, keep = _host_csr(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    snk = np.ascontiguousarray(sinks, dtype=np.int32)
    if src.shape != snk.shape:
        raise ValueError("sources and sinks must have the same length")
    k = int(src.shape[0])
    value = ctypes.c_int64(0)
    flow = np.zeros(max(csr.E, 1), np.int32) if want_flow else None
    side = np.zeros(max(g.V, 1), np.uint8) if want_side else None
    st = wbpr_stats()
    rc = lib.wbpr_solve_multi(ctx, ctypes.byref(csr), k, src.ctypes.data if k else None,
                              snk.ctypes.data if k else None, ctypes.addressof(value),
                              flow.ctypes.data if flow is not None else None,
                              side.ctypes.data if side is not None else None, ctypes.byref(st))
    if return_code:
        return rc
    _check(rc)
    return Result(int(value.value), flow[: csr.E] if flow is not None else None,
                  side[: g.V] if side is not None else None, st.as_dict())


def wbpr_solve_device(ctx: int, V: int, E: int, row_ptr_ptr: int, col_ptr: int, cap_ptr: int, s: int, t: int,
                      stream: int, value_ptr: int, flow_ptr: int | None, side_ptr: int | None) -> dict:
    """Solve from device pointers (e.g. torch tensor data_ptr()); returns the stats dict."""
    lib = load_library()
    g = wbpr_csr(V, E, row_ptr_ptr, col_ptr, cap_ptr)
    st = wbpr_stats()
    _check(lib.wbpr_solve_device(ctx, ctypes.byref(g), s, t, stream or None, value_ptr, flow_ptr or None,
                                 side_ptr or None, ctypes.byref(st)))
    return st.as_dict()


def wbpr_solve_device_noalloc(ctx: int, V: int, E: int, row_ptr_ptr: int, col_ptr: int, cap_ptr: int, s: int,
                              t: int, stream: int, value_ptr: int, flow_ptr: int | None,
                              side_ptr: int | None) -> dict:
    """wbpr_solve_device that allocates no device memory (the library's static
    scratch array); returns the stats dict."""
    lib = load_library()
    g = wbpr_csr(V, E, row_ptr_ptr, col_ptr, cap_ptr)
    st = wbpr_stats()
    _check(lib.wbpr_solve_device_noalloc(ctx, ctypes.byref(g), s, t, stream or None, value_ptr, flow_ptr or None,
                                         side_ptr or None, ctypes.byref(st)))
    return st.as_dict()


@dataclass
class BatchResult:
    values: np.ndarray           # int64[n]
    flows: list | None           # n arrays int32[E_i]
    sides: list | None           # n arrays uint8[V_i]
    stats: dict
    status: np.ndarray | None = None  # int32[n] per-instance codes (per_instance=True)


def wbpr_solve_batch(ctx: int, graphs, want_flow: bool = True, want_side: bool = True,
                     return_code: bool = False, per_instance: bool = False):
    """Batched solve from host graphs (objects with V, row_ptr, col, cap, s, t).
    per_instance: invalid instances get their own status code (and value 0)
    instead of failing the call."""
    lib = load_library()
    n = len(graphs)
    keep = []
    arr = (wbpr_csr * n)()
    for i, g in enumerate(graphs):
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(g.col, dtype=np.int32)
        k = np.ascontiguousarray(g.cap, dtype=np.int32)
        keep += [rp, c, k]
        E = int(c.shape[0])
        arr[i] = wbpr_csr(g.V, E, rp.ctypes.data, c.ctypes.data if E else None, k.ctypes.data if E else None)
    s = np.array([g.s for g in graphs], dtype=np.int32)
    t = np.array([g.t for g in graphs], dtype=np.int32)
    values = np.zeros(n, np.int64)
    flows = [np.zeros(max(int(np.asarray(g.col).shape[0]), 1), np.int32) for g in graphs] if want_flow else None
    sides = [np.zeros(g.V, np.uint8) for g in graphs] if want_side else None
    fp = (ctypes.c_void_p * n)(*[f.ctypes.data for f in flows]) if flows is not None else None
    sp = (ctypes.c_void_p * n)(*[x.ctypes.data for x in sides]) if sides is not None else None
    st = wbpr_stats()
    status = np.zeros(n, np.int32) if per_instance else None
    rc = lib.wbpr_solve_batch(ctx, n, arr, s.ctypes.data, t.ctypes.data, values.ctypes.data,
                              ctypes.cast(fp, ctypes.c_void_p) if fp is not None else None,
                              ctypes.cast(sp, ctypes.c_void_p) if sp is not None else None, ctypes.byref(st),
                              status.ctypes.data if status is not None else None)
    if return_code:
        return rc
    _check(rc)
    if flows is not None:
        flows = [f[: int(np.asarray(g.col).shape[0])] for f, g in zip(flows, graphs)]
    return BatchResult(values, flows, sides, st.as_dict(), status)


def wbpr_solve_batch_device(ctx: int, V, E, s, t, row_ptr_ptr: int, col_ptr: int, cap_ptr: int, stream: int,
                            values_ptr: int, flows_ptr: int | None, sides_ptr: int | None, status=None) -> dict:
    """Batched solve from packed device arrays; V, E, s, t are host sequences.
    status: optional host int32 numpy array [n] for per-instance codes."""
    lib = load_library()
    n = len(V)
    Va = np.ascontiguousarray(V, dtype=np.int32)
    Ea = np.ascontiguousarray(E, dtype=np.int64)
    sa = np.ascontiguousarray(s, dtype=np.int32)
    ta = np.ascontiguousarray(t, dtype=np.int32)
    st = wbpr_stats()
    _check(lib.wbpr_solve_batch_device(ctx, n, Va.ctypes.data, Ea.ctypes.data, sa.ctypes.data, ta.ctypes.data,
                                       row_ptr_ptr, col_ptr or None, cap_ptr or None, stream or None, values_ptr,
                                       flows_ptr or None, sides_ptr or None, ctypes.byref(st),
                                       status.ctypes.data if status is not None else None))
    return st.as_dict()


class Solver:
    """Context-owning convenience wrapper around the C ABI."""

    def __init__(self, device: int = 0, **options):
        self.ctx = wbpr_ctx_create(device, **options)
        _live_solvers.add(self)

    def set_options(self, **options):
        wbpr_ctx_set_options(self.ctx, **options)

    def solve(self, g, want_flow: bool = True, want_side: bool = True) -> Result:
        return wbpr_solve(self.ctx, g.V, g.row_ptr, g.col, g.cap, g.s, g.t, want_flow, want_side)

    def autotune(self, g, max_trials: int = 0, include_full_scan: bool = False):
        """(best options as a dict, best solve ms); also remembered by the context."""
        lib = load_library()
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(g.col, dtype=np.int32)
        k = np.ascontiguousarray(g.cap, dtype=np.int32)
        E = int(c.shape[0])
        csr = wbpr_csr(g.V, E, rp.ctypes.data, c.ctypes.data if E else None, k.ctypes.data if E else None)
        best = wbpr_options()
        ms = ctypes.c_double()
        _check(lib.wbpr_autotune(self.ctx, ctypes.byref(csr), g.s, g.t, max_trials, int(include_full_scan),
                                 ctypes.byref(best), ctypes.byref(ms)))
        return {name: getattr(best, name) for name, _ in best._fields_}, ms.value

    def bfs_farthest(self, g, sources):
        return wbpr_bfs_farthest(self.ctx, g, sources)

    def pick_terminals(self, g, k: int, seed: int = 1):
        return wbpr_pick_terminals(self.ctx, g, k, seed)

    def solve_multi(self, g, sources, sinks, want_flow: bool = True, want_side: bool = True) -> Result:
        return wbpr_solve_multi(self.ctx, g, sources, sinks, want_flow, want_side)

    def wave_trace(self) -> np.ndarray:
        """Per-wave records of the last solve (needs wave_trace=1): an int64
        array of shape (n, 5) with columns sweep, kernel (0 short-row tiles,
        1 medium rows, 2 first chunks, 3 further chunks), ticks of the 100 MHz
        device clock, arc scans, items (vertices or chunk tasks)."""
        lib = load_library()
        n = ctypes.c_int64()
        _check(lib.wbpr_wave_trace(self.ctx, None, 0, ctypes.byref(n)))
        rec = np.zeros((max(n.value, 1), 4), np.int32)
        _check(lib.wbpr_wave_trace(self.ctx, rec.ctypes.data, n.value, ctypes.byref(n)))
        rec = rec[: n.value].astype(np.int64)
        return np.stack([rec[:, 0] >> 2, rec[:, 0] & 3, rec[:, 1], rec[:, 2], rec[:, 3]], axis=1)

    def solve_batch(self, graphs, want_flow: bool = True, want_side: bool = True,
                    per_instance: bool = False) -> BatchResult:
        return wbpr_solve_batch(self.ctx, graphs, want_flow, want_side, per_instance=per_instance)

    def solve_tensors(self, V, row_ptr, col, cap, s, t, value, flow=None, side=None, stream=None) -> dict:
        """Device-resident solve on torch tensors (torch supplies the memory).

        The solve is ordered after the work queued on ``stream`` (default:
        torch's current stream on the tensors' device) and later work on that
        stream sees the outputs; the call returns with them written."""
        import torch

        for x in (row_ptr, col, cap, value, flow, side):
            if x is not None and (not x.is_cuda or not x.is_contiguous()):
                raise ValueError("tensors must be contiguous device tensors")
        if stream is None:
            stream = torch.cuda.current_stream(row_ptr.device)
        return wbpr_solve_device(self.ctx, V, int(col.shape[0]), row_ptr.data_ptr(), col.data_ptr(),
                                 cap.data_ptr(), s, t, int(stream.cuda_stream), value.data_ptr(),
                                 flow.data_ptr() if flow is not None else None,
                                 side.data_ptr() if side is not None else None)

    def close(self):
        if self.ctx:
            wbpr_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wbpr_server_footprint(V: int, E: int) -> int:
    out = ctypes.c_int64()
    _check(load_library().wbpr_server_footprint(V, E, ctypes.byref(out)))
    return out.value


@dataclass
class ServedResult:
    ticket: int
    status: int
    value: int
    flow: np.ndarray | None
    side: np.ndarray | None
    latency_ms: float
    queue_ms: float


class Server:
    """Continuous-batching server on a context's device (thread-safe submit/wait)."""

    def __init__(self, solver: "Solver", hbm_budget_bytes: int = 0, max_slots: int = 0, arcs_per_vertex: int = 0,
                 want_flows: bool = True, want_sides: bool = True, max_admit: int = 0):
        lib = load_library()
        o = wbpr_server_options()
        o.hbm_budget_bytes = hbm_budget_bytes
        o.max_slots = max_slots
        o.arcs_per_vertex = arcs_per_vertex
        o.want_flows = int(want_flows)
        o.want_sides = int(want_sides)
        o.max_admit = max_admit
        h = ctypes.c_void_p()
        _check(lib.wbpr_server_create(solver.ctx, ctypes.byref(o), ctypes.byref(h)))
        self.h = h.value
        self._solver = solver  # the context must outlive the server
        _live_servers.add(self)

    def submit(self, g, return_code: bool = False):
        lib = load_library()
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(g.col, dtype=np.int32)
        k = np.ascontiguousarray(g.cap, dtype=np.int32)
        E = int(c.shape[0])
        csr = wbpr_csr(g.V, E, rp.ctypes.data, c.ctypes.data if E else None, k.ctypes.data if E else None)
        tk = ctypes.c_uint64()
        rc = lib.wbpr_server_submit(self.h, ctypes.byref(csr), g.s, g.t, ctypes.byref(tk))
        if return_code:
            return rc, tk.value
        _check(rc)
        return tk.value

    def _take(self, r: wbpr_result) -> ServedResult:
        flow = np.ctypeslib.as_array(r.arc_flow, shape=(r.E,)).copy() if r.arc_flow else None
        side = np.ctypeslib.as_array(r.cut_side, shape=(r.V,)).copy() if r.cut_side else None
        out = ServedResult(r.ticket, r.status, r.value, flow, side, r.latency_ms, r.queue_ms)
        load_library().wbpr_result_free(ctypes.byref(r))
        return out

    def poll(self, ticket: int):
        """ServedResult when ready, None while pending."""
        r = wbpr_result()
        rc = load_library().wbpr_server_poll(self.h, ticket, ctypes.byref(r))
        if rc == WBPR_EAGAIN:
            return None
        _check(rc)
        return self._take(r)

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = wbpr_result()
        rc = load_library().wbpr_server_wait(self.h, ticket, timeout_ms, ctypes.byref(r))
        if rc == WBPR_EAGAIN:
            return None
        _check(rc)
        return self._take(r)

    def stats(self) -> dict:
        st = wbpr_server_stats()
        _check(load_library().wbpr_server_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self.h:
            load_library().wbpr_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UploadedGraph:
    """A graph whose residual form stays on the device: many (s, t) solves
    without rebuilding it (wbpr_graph_upload / wbpr_graph_solve)."""

    def __init__(self, solver: "Solver", g):
        lib = load_library()
        self._rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        self._col = np.ascontiguousarray(g.col, dtype=np.int32)
        self._cap = np.ascontiguousarray(g.cap, dtype=np.int32)
        self.V = int(g.V)
        self.E = int(self._col.shape[0])
        csr = wbpr_csr(self.V, self.E, self._rp.ctypes.data, self._col.ctypes.data if self.E else None,
                       self._cap.ctypes.data if self.E else None)
        h = ctypes.c_void_p()
        _check(lib.wbpr_graph_upload(solver.ctx, ctypes.byref(csr), ctypes.byref(h)))
        self.h = h.value
        del self._rp, self._col, self._cap  # the library copied them
        _live_graphs.add(self)

    def solve(self, s: int, t: int, want_flow: bool = True, want_side: bool = True, return_code: bool = False):
        lib = load_library()
        value = ctypes.c_int64()
        flow = np.zeros(max(self.E, 1), np.int32) if want_flow else None
        side = np.zeros(self.V, np.uint8) if want_side else None
        st = wbpr_stats()
        rc = lib.wbpr_graph_solve(self.h, s, t, ctypes.byref(value), flow.ctypes.data if flow is not None else None,
                                  side.ctypes.data if side is not None else None, ctypes.byref(st))
        if return_code:
            return rc
        _check(rc)
        return Result(value.value, flow[: self.E] if flow is not None else None, side, st.as_dict())

    def close(self):
        if self.h:
            load_library().wbpr_graph_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
