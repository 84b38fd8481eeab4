"""Seeded synthetic graphs as undirected CSR (int64 offsets, int32 columns).

Input preparation only: nothing here performs any part of the traversal.  The
generators live in ``graphgen.cpp`` (host C++, OpenMP) and are reached through
ctypes; every draw comes from a counter-based SplitMix64 stream keyed by
(seed, stream, index), so a graph is a pure function of its parameters.

Workload shapes follow the paper's evaluation graphs in spirit (scale-free
social/web graphs, meshes, random graphs); the paper's own KONECT collection
is not used, synthetic graphs of these families stand in for it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile graphgen.cpp into libgraphgen.so next to it (host g++)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [i32, i32, dbl, dbl, dbl, u64, i32]
    lib.gg_grid.restype = vp
    lib.gg_grid.argtypes = [i32, i32, dbl, u64]
    lib.gg_chung_lu.restype = vp
    lib.gg_chung_lu.argtypes = [i64, dbl, dbl, u64, i32]
    lib.gg_erdos_renyi.restype = vp
    lib.gg_erdos_renyi.argtypes = [i64, i64, u64]
    lib.gg_from_edges.restype = vp
    lib.gg_from_edges.argtypes = [i64, i64, vp, vp, i32, i32, i32]
    lib.gg_n.restype = i64
    lib.gg_n.argtypes = [vp]
    lib.gg_nnz.restype = i64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_pick_sources.restype = i64
    lib.gg_pick_sources.argtypes = [i64, vp, i64, u64, vp]
    lib.gg_ctr_rand.restype = u64
    lib.gg_ctr_rand.argtypes = [u64, u64, u64]
    _lib = lib
    return lib


@dataclass
class CSR:
    """Undirected graph: row ``v`` holds ``cols[offs[v]:offs[v+1]]`` ascending."""

    offs: np.ndarray
    cols: np.ndarray
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offs.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.cols.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offs)


def _take(h, name, params) -> CSR:
    lib = _load()
    if not h:
        raise ValueError("graph generator rejected parameters %r" % (params,))
    try:
        n, nnz = lib.gg_n(h), lib.gg_nnz(h)
        offs = np.empty(n + 1, dtype=np.int64)
        cols = np.empty(nnz, dtype=np.int32)
        lib.gg_copy(h, offs.ctypes.data, cols.ctypes.data)
    finally:
        lib.gg_free(h)
    return CSR(offs, cols, name, dict(params))


def rmat(scale: int, edgefactor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, relabel: bool = True) -> CSR:
    """R-MAT graph: 2**scale vertices, edgefactor*2**scale generated pairs
    before symmetrisation, loop and repeat removal."""
    p = dict(family="rmat", scale=scale, edgefactor=edgefactor, a=a, b=b, c=c, seed=seed,
             relabel=bool(relabel))
    h = _load().gg_rmat(scale, edgefactor, a, b, c, seed, int(relabel))
    return _take(h, "rmat%d_ef%d_s%d" % (scale, edgefactor, seed), p)


def grid(rows: int, cols: int, delete_frac: float = 0.0, seed: int = 3) -> CSR:
    """rows x cols four-neighbour grid with floor(delete_frac*m) edges removed."""
    p = dict(family="grid", rows=rows, cols=cols, delete_frac=delete_frac, seed=seed)
    h = _load().gg_grid(rows, cols, delete_frac, seed)
    return _take(h, "grid%dx%d_del%g_s%d" % (rows, cols, delete_frac, seed), p)


def chung_lu(n: int, gamma: float = 2.1, mean_degree: float = 20.0, seed: int = 4,
             relabel: bool = True) -> CSR:
    """Chung-Lu power-law graph (expected-degree cap sqrt(n*mean_degree))."""
    p = dict(family="chung_lu", n=n, gamma=gamma, mean_degree=mean_degree, seed=seed,
             relabel=bool(relabel))
    h = _load().gg_chung_lu(n, gamma, mean_degree, seed, int(relabel))
    return _take(h, "chunglu%d_g%g_d%g_s%d" % (n, gamma, mean_degree, seed), p)


def erdos_renyi(n: int, m: int, seed: int = 5) -> CSR:
    """G(n, m) with m uniform pairs drawn with replacement (repeats dropped)."""
    p = dict(family="erdos_renyi", n=n, m=m, seed=seed)
    h = _load().gg_erdos_renyi(n, m, seed)
    return _take(h, "er%d_m%d_s%d" % (n, m, seed), p)


def from_edges(n: int, src, dst, symmetrize: bool = True, drop_loops: bool = True,
               dedup: bool = True, name: str = "edges") -> CSR:
    """CSR of an explicit pair list (rows sorted; loops/repeats optionally kept)."""
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    d = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    h = _load().gg_from_edges(n, s.shape[0], s.ctypes.data, d.ctypes.data, int(symmetrize),
                              int(drop_loops), int(dedup))
    return _take(h, name, dict(family="edges", n=n, m=int(s.shape[0])))


def pick_sources(g: CSR, k: int, seed: int) -> np.ndarray:
    """k distinct seeded sources among vertices of degree > 0."""
    out = np.empty(max(k, 0), dtype=np.int32)
    offs = np.ascontiguousarray(g.offs, dtype=np.int64)
    got = _load().gg_pick_sources(g.n, offs.ctypes.data, k, seed, out.ctypes.data)
    if got < 0:
        raise ValueError("bad arguments to pick_sources")
    return out[:got]


def ctr_rand(seed: int, stream: int, idx: int) -> int:
    return int(_load().gg_ctr_rand(seed, stream, idx))


# Named workloads (sizes, families and seeds used by the tests and the bench).
def workload(name: str) -> CSR:
    if name == "rmat10":
        return rmat(10, 16, seed=1)
    if name == "rmat22":
        return rmat(22, 16, seed=2)
    if name == "grid2048_del5":
        return grid(2048, 2048, 0.05, seed=3)
    if name == "chunglu23":
        return chung_lu(1 << 23, 2.1, 20.0, seed=4)
    if name == "er22":
        return erdos_renyi(1 << 22, 4 << 22, seed=5)
    if name == "rmat20":
        return rmat(20, 16, seed=6)
    raise KeyError(name)


WORKLOAD_SOURCES = {"rmat10": (1, 101), "rmat22": (64, 102), "grid2048_del5": (32, 103),
                    "chunglu23": (32, 104), "er22": (32, 105), "rmat20": (1024, 106)}
