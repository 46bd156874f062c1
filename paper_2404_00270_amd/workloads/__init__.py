"""Seeded synthetic max-flow workloads (input generation only).

The graphs stand in for the paper's evaluation inputs (section 4: SNAP and
DIMACS max-flow graphs, KONECT bipartite matching graphs), which are not
available here.  Every graph is a CSR (``row_ptr`` int64[V+1], ``col``
int32[E], ``cap`` int32[E]) plus a source and a sink.  The generators live in
``wbgen.c``; this module only marshals their output into numpy arrays.
Nothing here computes flows: both the CPU oracle and the HIP solver consume
these arrays.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwbgen.so")
SRC_PATH = os.path.join(_HERE, "wbgen.c")


class _CGraph(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_int32),
        ("E", ctypes.c_int64),
        ("rp", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("cap", ctypes.POINTER(ctypes.c_int32)),
        ("s", ctypes.c_int32),
        ("t", ctypes.c_int32),
    ]


@dataclass
class Graph:
    """A directed graph in CSR with integer capacities, a source and a sink."""

    V: int
    row_ptr: np.ndarray  # int64[V+1]
    col: np.ndarray      # int32[E]
    cap: np.ndarray      # int32[E]
    s: int
    t: int
    name: str = ""

    @property
    def E(self) -> int:
        return int(self.col.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.array([self.V, self.s, self.t], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.cap, dtype=np.int32).tobytes())
        return h.hexdigest()


def build_lib(force: bool = False) -> str:
    """Compile wbgen.c into libwbgen.so next to it (plain gcc)."""
    import subprocess

    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_CGraph)
        lib.wbgen_random.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P]
        lib.wbgen_multi.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, P]
        lib.wbgen_bipartite.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, P]
        lib.wbgen_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P]
        lib.wbgen_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, P]
        lib.wbgen_batch_instance.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_uint64, P]
        for fn in ("wbgen_random", "wbgen_multi", "wbgen_bipartite", "wbgen_rmat", "wbgen_grid", "wbgen_batch_instance"):
            getattr(lib, fn).restype = ctypes.c_int
        lib.wbgen_free.argtypes = [P]
        lib.wbgen_free.restype = None
        _lib = lib
    return _lib


def _take(cg: _CGraph, name: str) -> Graph:
    lib = _load()
    V, E = cg.V, cg.E
    rp = np.ctypeslib.as_array(cg.rp, shape=(V + 1,)).copy()
    if E > 0:
        col = np.ctypeslib.as_array(cg.col, shape=(E,)).copy()
        cap = np.ctypeslib.as_array(cg.cap, shape=(E,)).copy()
    else:
        col = np.zeros(0, np.int32)
        cap = np.zeros(0, np.int32)
    g = Graph(V=V, row_ptr=rp, col=col, cap=cap, s=int(cg.s), t=int(cg.t), name=name)
    lib.wbgen_free(ctypes.byref(cg))
    return g


def _call(fn, name, *args) -> Graph:
    cg = _CGraph()
    rc = fn(*args, ctypes.byref(cg))
    if rc != 0:
        raise ValueError(f"workload generator {name} failed (rc={rc})")
    return _take(cg, name)


def random_graph(V: int, E: int, cmin: int = 1, cmax: int = 100, seed: int = 1) -> Graph:
    """E distinct uniform arcs (no self-loops), caps uniform on [cmin,cmax]; s=0, t=V-1."""
    lib = _load()
    return _call(lib.wbgen_random, f"random(V={V},E={E},seed={seed})", V, E, cmin, cmax, seed)


def multigraph(V: int, E: int, cmax: int = 20, seed: int = 1) -> Graph:
    """Uniform endpoints with parallel/antiparallel arcs and self-loops; caps on [0,cmax]."""
    lib = _load()
    return _call(lib.wbgen_multi, f"multi(V={V},E={E},seed={seed})", V, E, cmax, seed)


def bipartite(L: int, R: int, narcs: int, expo: float = 2.1, seed: int = 2) -> Graph:
    """Bipartite matching as max flow: uniform left ends, Zipf(expo) right ends, unit caps."""
    lib = _load()
    return _call(lib.wbgen_bipartite, f"bipartite(L={L},R={R},arcs={narcs},seed={seed})", L, R, narcs, expo, seed)


def rmat(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         cmin: int = 1, cmax: int = 1000, seed: int = 3) -> Graph:
    """R-MAT power-law graph, permuted ids, duplicates/self-loops removed."""
    lib = _load()
    return _call(lib.wbgen_rmat, f"rmat(scale={scale},ef={ef},seed={seed})", scale, ef, a, b, c, cmin, cmax, seed)


def grid(W: int, H: int, sigma: float = 0.1, sigma_s: float = 1.0, seed: int = 4) -> Graph:
    """Vision-style 4-connected grid cut with s/t links to every pixel."""
    lib = _load()
    return _call(lib.wbgen_grid, f"grid({W}x{H},seed={seed})", W, H, sigma, sigma_s, seed)


BATCH_SEED_BASE = 5 << 32


def batch_instance(i: int, vmin: int = 256, vmax: int = 65536, deg: int = 8,
                   cmin: int = 1, cmax: int = 100, seed_base: int = BATCH_SEED_BASE) -> Graph:
    """Instance i of the batched stream: log-uniform V, deg*V distinct uniform arcs."""
    lib = _load()
    return _call(lib.wbgen_batch_instance, f"batch[{i}]", vmin, vmax, deg, cmin, cmax, seed_base + i)


# The five evaluation workloads, sized as the paper-shaped configurations.
def config_plain(seed: int = 1) -> Graph:
    """V=1,000, 8,000 distinct uniform arcs, caps U[1,100], s=0, t=999."""
    g = random_graph(1000, 8000, 1, 100, seed)
    g.name = "plain-V1000-E8000"
    return g


def config_bipartite(seed: int = 2, L: int = 50_000, R: int = 50_000, narcs: int = 1_000_000) -> Graph:
    """50k+50k bipartite, 1M Zipf(2.1) arcs, super-source/sink, unit caps."""
    g = bipartite(L, R, narcs, 2.1, seed)
    g.name = f"bipartite-zipf-{L}x{R}-{narcs}"
    return g


def config_rmat(seed: int = 3, scale: int = 22) -> Graph:
    """R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), caps U[1,1000]."""
    g = rmat(scale, 16, 0.57, 0.19, 0.19, 1, 1000, seed)
    g.name = f"rmat-s{scale}-ef16"
    return g


def config_grid(seed: int = 4, W: int = 2048, H: int = 2048) -> Graph:
    """2048x2048 grid cut, sigma=0.1 n-links, t-links U{0..255}."""
    g = grid(W, H, 0.1, 1.0, seed)
    g.name = f"grid-{W}x{H}"
    return g


WORKLOADS = {
    "plain": config_plain,
    "bipartite": config_bipartite,
    "rmat": config_rmat,
    "grid": config_grid,
}


def from_arcs(V: int, arcs, s: int, t: int, name: str = "") -> Graph:
    """CSR from an explicit arc list [(u, v, cap), ...]; arcs keep list order inside a row."""
    arcs = list(arcs)
    E = len(arcs)
    if E:
        u = np.array([a[0] for a in arcs], dtype=np.int64)
        v = np.array([a[1] for a in arcs], dtype=np.int32)
        c = np.array([a[2] for a in arcs], dtype=np.int32)
        order = np.argsort(u, kind="stable")
        u, v, c = u[order], v[order], c[order]
        rp = np.zeros(V + 1, np.int64)
        np.add.at(rp, u + 1, 1)
        rp = np.cumsum(rp).astype(np.int64)
    else:
        v = np.zeros(0, np.int32)
        c = np.zeros(0, np.int32)
        rp = np.zeros(V + 1, np.int64)
    return Graph(V=V, row_ptr=rp, col=v, cap=c, s=s, t=t, name=name)


def arc_sources(g: Graph) -> np.ndarray:
    """Tail vertex of every arc (int32[E])."""
    return np.repeat(np.arange(g.V, dtype=np.int32), np.diff(g.row_ptr))
