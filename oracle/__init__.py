"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded max-flow solvers (Dinic; two-phase FIFO push-relabel
with global relabelling and the gap heuristic) and an independent flow
certificate, all in ``oracle.c``.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the HIP product path
never does, and this package imports nothing from it.

Functions take plain numpy arrays: ``V`` vertices, CSR ``row_ptr``
(int64[V+1]), ``col`` (int32[E]), ``cap`` (int32[E]), source ``s`` and sink
``t``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (idempotent unless forced)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        solver_args = [i32, i64, vp, vp, vp, i32, i32, vp, vp, vp]
        for fn in ("orc_dinic", "orc_fifo_pr"):
            getattr(lib, fn).argtypes = solver_args
            getattr(lib, fn).restype = ctypes.c_int
        lib.orc_check.argtypes = [i32, i64, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp]
        lib.orc_check.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _prep(V, row_ptr, col, cap):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    k = np.ascontiguousarray(cap, dtype=np.int32)
    if rp.shape != (V + 1,) or c.shape != k.shape:
        raise ValueError("bad CSR shapes")
    # keep 1-element buffers for empty arc lists so pointers are valid
    if c.size == 0:
        c = np.zeros(1, np.int32)
        k = np.zeros(1, np.int32)
    return rp, c, k


@dataclass
class OracleResult:
    value: int
    flow: np.ndarray  # int32[E]
    arc_scans: int


def _solve(fn_name, V, row_ptr, col, cap, s, t) -> OracleResult:
    lib = _load()
    E = int(np.asarray(col).shape[0])
    rp, c, k = _prep(V, row_ptr, col, cap)
    flow = np.zeros(max(E, 1), np.int32)
    val = ctypes.c_int64(0)
    scans = ctypes.c_int64(0)
    rc = getattr(lib, fn_name)(V, E, _ptr(rp), _ptr(c), _ptr(k), s, t,
                               ctypes.addressof(val), _ptr(flow), ctypes.addressof(scans))
    if rc != 0:
        raise RuntimeError(f"{fn_name} failed with rc={rc}")
    return OracleResult(int(val.value), flow[:E].copy(), int(scans.value))


def dinic(V, row_ptr, col, cap, s, t) -> OracleResult:
    """Dinic: level graph + blocking flow (maximum flow value and one max flow)."""
    return _solve("orc_dinic", V, row_ptr, col, cap, s, t)


def fifo_pr(V, row_ptr, col, cap, s, t) -> OracleResult:
    """Two-phase FIFO push-relabel (maximum flow value and one max flow)."""
    return _solve("orc_fifo_pr", V, row_ptr, col, cap, s, t)


@dataclass
class CheckResult:
    code: int          # 0 feasible, 1 capacity violated, 2 conservation violated
    bad: int           # offending arc (code 1) or vertex (code 2)
    value: int         # flow value (net out of s)
    side: np.ndarray   # uint8[V]: 1 iff v reaches t in the residual graph
    cut_capacity: int  # capacity of the cut side 0 -> side 1

    @property
    def feasible(self) -> bool:
        return self.code == 0

    def is_maximum(self, s: int) -> bool:
        """Feasible, value equals the cut capacity, and s is on the source side."""
        return self.code == 0 and self.value == self.cut_capacity and int(self.side[s]) == 0


def check(V, row_ptr, col, cap, s, t, flow) -> CheckResult:
    """Certificate for a flow: feasibility, value, canonical sink side, cut capacity."""
    lib = _load()
    E = int(np.asarray(col).shape[0])
    rp, c, k = _prep(V, row_ptr, col, cap)
    f = np.ascontiguousarray(flow, dtype=np.int32)
    if f.shape != (E,):
        raise ValueError("flow must have one entry per arc")
    if f.size == 0:
        f = np.zeros(1, np.int32)
    side = np.zeros(V, np.uint8)
    val = ctypes.c_int64(0)
    cut = ctypes.c_int64(0)
    bad = ctypes.c_int64(-1)
    rc = lib.orc_check(V, E, _ptr(rp), _ptr(c), _ptr(k), s, t, _ptr(f), ctypes.addressof(val),
                       _ptr(side), ctypes.addressof(cut), ctypes.addressof(bad))
    if rc < 0:
        raise RuntimeError(f"orc_check failed with rc={rc}")
    return CheckResult(rc, int(bad.value), int(val.value), side, int(cut.value))


def reference(V, row_ptr, col, cap, s, t):
    """Oracle answer: value (both solvers must agree), canonical sink side and cut capacity."""
    a = dinic(V, row_ptr, col, cap, s, t)
    b = fifo_pr(V, row_ptr, col, cap, s, t)
    if a.value != b.value:
        raise RuntimeError(f"oracle disagreement: dinic={a.value} fifo_pr={b.value}")
    ca = check(V, row_ptr, col, cap, s, t, a.flow)
    if not ca.feasible or ca.value != a.value or ca.cut_capacity != a.value:
        raise RuntimeError("oracle flow failed its own certificate")
    return a.value, ca.side, ca.cut_capacity
