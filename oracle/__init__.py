"""CPU oracle for the level-switched BFS library -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
imports nothing from the GPU library (the seeded input generators are the one
shared module, and they hold none of the traversal's arithmetic).

Contents
  * ``bfs``           -- plain single-threaded FIFO BFS in C (``bfs_oracle.c``):
                         hop-distance levels, one valid parent per vertex, the
                         per-depth vertex and degree histograms.
  * ``components``    -- weakly connected components in C (disjoint-set
                         forest), labelled by each component's smallest id.
  * ``msbfs_levels``  -- the multi-source result: one ``bfs`` per source,
                         stored as int8 with the 127 cap as a range error.
  * ``checks``        -- Graph500-style invariants and connected components.
  * ``features``      -- the per-level feature vector from its definition
                         (Section IV-A, feature list; Section IV-B, best model).
  * ``tree``          -- decision-tree prediction with the paper's rule for an
                         undecided ("unknown") leaf (Section IV-A, last
                         paragraphs).
  * ``schedule``      -- best-per-level ("optimal traversal") arithmetic
                         (Section IV-B, first paragraph).

Pins (tests marked not-gpu): brute-force all-pairs shortest paths on tiny
graphs, scipy/networkx shortest paths, closed forms (paths, cycles, stars,
complete and complete bipartite graphs, grids, binary trees, hypercubes, the
Petersen graph), invariants, and sklearn's own tree prediction.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", src, "-o", tmp], check=True)
        os.replace(tmp, out)
    return out


def load(path: str = _LIB):
    lib = ctypes.CDLL(path)
    lib.oracle_bfs.restype = ctypes.c_int64
    lib.oracle_bfs.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_components.restype = ctypes.c_int64
    lib.oracle_components.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load(_LIB)
    return _lib


def bfs(offs, cols, source: int, lib=None):
    """Hop-distance BFS from ``source``.

    Returns ``(level int32[n], parent int32[n], hist int64[D], ehist int64[D])``
    where D is the eccentricity of ``source`` plus one; ``hist[d]`` counts
    the vertices at depth d and ``ehist[d]`` sums their degrees.
    """
    lib = lib or _get()
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = offs.shape[0] - 1
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    hist = np.empty(n, dtype=np.int64)
    ehist = np.empty(n, dtype=np.int64)
    nd = lib.oracle_bfs(n, offs.ctypes.data, cols.ctypes.data, int(source), level.ctypes.data,
                        parent.ctypes.data, hist.ctypes.data, ehist.ctypes.data)
    if nd < 0:
        raise ValueError("oracle_bfs rejected its arguments (n=%d, source=%d)" % (n, source))
    return level, parent, hist[:nd].copy(), ehist[:nd].copy()


def levels(offs, cols, source: int) -> np.ndarray:
    return bfs(offs, cols, source)[0]


INT8_CAP = 127


def msbfs_levels(offs, cols, sources, cap: int = INT8_CAP):
    """Levels of many sources as int8 ``[len(sources)][n]`` (-1 = unreached).

    Returns ``(levels, in_range)``; ``in_range`` is False when some source
    reaches a depth above ``cap`` -- such a result cannot be stored in int8
    and must be reported as a range error, never truncated.
    """
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    n = offs.shape[0] - 1
    out = np.empty((len(sources), n), dtype=np.int8)
    ok = True
    for i, s in enumerate(sources):
        lv = levels(offs, cols, int(s))
        if lv.max() > cap:
            ok = False
        out[i] = np.where(lv > cap, cap, lv).astype(np.int8)
    return out, ok


def components(offs, cols, lib=None):
    """Weakly connected components (``bfs_oracle.c``, disjoint-set forest):
    ``(label int32[n], count)``, ``label[v]`` the smallest vertex id of the
    component of v, every arc joining its ends whatever its direction."""
    lib = lib or _get()
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = offs.shape[0] - 1
    label = np.empty(n, dtype=np.int32)
    c = lib.oracle_components(n, offs.ctypes.data, cols.ctypes.data, label.ctypes.data)
    if c < 0:
        raise ValueError("oracle_components rejected its arguments (n=%d)" % n)
    return label, int(c)


def component_edges(offs, level) -> int:
    """Undirected edges inside the traversed component: half the degree sum of
    reached vertices (the TEPS numerator)."""
    deg = np.diff(np.asarray(offs, dtype=np.int64))
    return int(deg[np.asarray(level) >= 0].sum() // 2)
