"""Algorithmic HBM bytes of one BFS level, per kernel family, and TEPS counts.

Measurement arithmetic for the roofline: what each expansion kernel must move
at level d, counted at the granularity it accesses (4-byte ids and levels,
8-byte offsets, 64-bit bitmap words).  Computed exactly on the host from a
level array (the GPU's own output) and the sorted CSR of a symmetric graph;
the per-level counts come from one pass over the rows in C
(``csrc/traffic_model.cpp``, OpenMP).

Terms (n_f = depth-d vertices, e_f = sum of their degrees, n_x = depth-(d+1)
vertices, nw = ceil(n/64) bitmap words):
  every kernel   nw*8 (zeroing the bitmap of the level after next)
                 + n_x*(4 level + 4 parent + 4 queue slot)
  top-down       + e_f*(4 column + 8 visited word) + n_x*8 (next-bitmap word)
    push_vertex, push_wave*: + n_f*(4 queue + 16 row offsets)
    push_edge:               + n_f*(4 queue + 16 row offsets + 8+8 scan and row
                               start written, 8+8+4 read back when staging tiles)
    vertex_scan:             + n*4 (every level read) + n_f*16
    edge_scan:               + nnz*4 (origin of every arc) + n*4 (its level,
                               read once per origin run)
    rev_edge_scan:           + nnz*4 (destination of every arc) + nw*8 (its
                               visited word, read once per run of a word)
  pull_bitmap    + nw*8 (visited words) + sum over unvisited v of
                 (16 head record + q_v*(4 column + 8 frontier word)
                  + 16 row offsets when v reads its row)
                 + 16 per word holding a discovery (visited and next words).
                 The probes start from the head: v probes its min(4, deg)
                 head neighbours; when none is in the frontier and the row
                 has at least four arcs, it reads its row bounds and probes
                 the row up to the first frontier neighbour (all of it when
                 none is).  On a skewed degree law (standard deviation above
                 the mean) the head is ranked -- the four neighbours of
                 largest degree among the first 256 arcs -- and the row is
                 probed from its start; otherwise the head is the first four
                 arcs and the row is probed past them.  q_v counts the probes.  Degree-0 vertices start visited (the search marks
                 them at init), so they cost only their visited bit.

``pull_bytes_literal`` is the pull formula exactly as the scope table writes
it -- (n/64)*8*3 for the visited, frontier and next words, 16 + p_v*12 for
every unvisited vertex including the degree-0 ones, p_v the neighbours in row
order up to the first one in the frontier, and n_x*12 -- reported beside the
model above.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PUSH_FAMILY = (0, 1, 2, 3, 4, 5)
PUSH_EDGE, PULL, VERTEX_SCAN, EDGE_SCAN, REV_EDGE_SCAN = 6, 7, 8, 9, 10
N_BASE = 11

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgswmodel.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build

            build.build_model()
        L = ctypes.CDLL(_LIB_PATH)
        L.tm_level_counts.restype = ctypes.c_int64
        L.tm_level_counts.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int64] + \
            [ctypes.c_void_p] * 4
        L.tm_head_counts.restype = ctypes.c_int64
        L.tm_head_counts.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int64] + \
            [ctypes.c_void_p] * 5 + [ctypes.c_int32]
        _lib = L
    return _lib


class Counts:
    """Per-depth counts of one source's BFS (see ``csrc/traffic_model.cpp``)."""

    def __init__(self, offs, cols, level, source: int, ranked=None):
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        self.ranked = head_is_ranked(offs) if ranked is None else bool(ranked)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        level = np.ascontiguousarray(level, dtype=np.int32)
        n = level.shape[0]
        cap = int(level.max()) + 2
        self.nf, self.ef, self.words, self.save = (np.zeros(cap, dtype=np.int64) for _ in range(4))
        D = _load().tm_level_counts(n, offs.ctypes.data, cols.ctypes.data, level.ctypes.data, cap,
                                    self.nf.ctypes.data, self.ef.ctypes.data, self.words.ctypes.data,
                                    self.save.ctypes.data)
        if D < 0:
            raise ValueError("level array deeper than its own maximum")
        self.D = int(D)
        self.n = n
        self.nnz = int(offs[-1])
        self.nw = (n + 63) // 64
        self.n_pos = int(np.count_nonzero(offs[1:] > offs[:-1]))  # vertices with arcs
        self.src_isolated = int(offs[source + 1] == offs[source])
        self.cum_nf = np.cumsum(self.nf)
        self.cum_ef = np.cumsum(self.ef)
        self.fcost, self.rowc, self.fsave, self.rsave = (np.zeros(cap, dtype=np.int64) for _ in range(4))
        tot = np.zeros(2, dtype=np.int64)
        if _load().tm_head_counts(n, offs.ctypes.data, cols.ctypes.data, level.ctypes.data, cap,
                                  self.fcost.ctypes.data, self.rowc.ctypes.data, self.fsave.ctypes.data,
                                  self.rsave.ctypes.data, tot.ctypes.data, int(self.ranked)) < 0:
            raise ValueError("level array deeper than its own maximum")
        self.full_total, self.row_total = int(tot[0]), int(tot[1])
        self.cum_fcost = np.cumsum(self.fcost)
        self.cum_rowc = np.cumsum(self.rowc)

    def at(self, a, d):
        return int(a[d]) if 0 <= d < a.shape[0] else 0

    def head_terms(self, d: int):
        """(probes, row reads) of a bottom-up level d starting from the head
        (ranked or the first arcs, as ``self.ranked`` says)."""
        probes = self.full_total - self.at(self.cum_fcost, d) - self.at(self.fsave, d)
        rows = self.row_total - self.at(self.cum_rowc, d) - self.at(self.rsave, d)
        return probes, rows

    def pull_terms(self, d: int):
        """(probes, unvisited vertices with arcs, unvisited vertices) at level d."""
        probes = self.nnz - self.at(self.cum_ef, d) - self.at(self.save, d)
        reached = self.at(self.cum_nf, d)
        unv_pos = self.n_pos - (reached - self.src_isolated)
        return probes, unv_pos, self.n - reached


def head_is_ranked(offs) -> bool:
    """Whether the library ranks the head of this graph: its out-degree
    standard deviation (population) is above the mean degree."""
    deg = np.diff(np.asarray(offs, dtype=np.int64))
    if deg.shape[0] == 0 or int(deg.sum()) == 0:
        return False
    return bool(deg.std() > deg.mean())


def component_edges(offs, level) -> int:
    """Undirected edges in the traversed component: half the reached degree sum."""
    deg = np.diff(np.asarray(offs, dtype=np.int64))
    return int(deg[np.asarray(level) >= 0].sum() // 2)


def level_sizes(offs, level):
    """(n_f[d], e_f[d]) for every depth d of a level array."""
    lv = np.asarray(level)
    deg = np.diff(np.asarray(offs, dtype=np.int64))
    r = lv >= 0
    D = int(lv.max()) + 1 if r.any() else 0
    nf = np.bincount(lv[r], minlength=D).astype(np.int64)
    ef = np.bincount(lv[r], weights=deg[r], minlength=D).astype(np.int64)
    return nf, ef


def level_bytes(kernel: int, c: Counts, d: int) -> int:
    """Algorithmic bytes of running ``kernel`` (a kernel id: the count
    variant does not change them) at level d (see module doc)."""
    k = kernel % N_BASE
    n_f, e_f, n_x = c.at(c.nf, d), c.at(c.ef, d), c.at(c.nf, d + 1)
    b = c.nw * 8 + n_x * 12
    if k == PULL:
        _, unv_pos, _ = c.pull_terms(d)
        probes, rows = c.head_terms(d)
        return b + c.nw * 8 + unv_pos * 16 + rows * 16 + probes * 12 + c.at(c.words, d + 1) * 16
    b += e_f * 12 + n_x * 8
    if k in PUSH_FAMILY:
        return b + n_f * 20
    if k == PUSH_EDGE:
        return b + n_f * (20 + 16 + 20)
    if k == VERTEX_SCAN:
        return b + c.n * 4 + n_f * 16
    if k == EDGE_SCAN:
        return b + c.nnz * 4 + c.n * 4
    if k == REV_EDGE_SCAN:
        return b + c.nnz * 4 + c.nw * 8
    raise ValueError("unknown kernel %r" % kernel)


def pull_bytes_literal(c: Counts, d: int) -> int:
    """The pull formula as the scope table writes it (degree-0 vertices
    counted as unvisited, 24 bytes per bitmap word)."""
    probes, _, unv_all = c.pull_terms(d)
    return c.nw * 8 * 3 + unv_all * 16 + probes * 12 + c.at(c.nf, d + 1) * 12


def pull_probes_reference(offs, cols, level, d: int, skip_isolated: bool = True):
    """(sum of p_v, unvisited count) for a pull at level d, by walking every
    unvisited row in numpy (slow; the check of ``Counts``)."""
    offs = np.asarray(offs, dtype=np.int64)
    lv = np.asarray(level)
    unvisited = (lv == -1) | (lv > d)
    if skip_isolated:
        unvisited &= offs[1:] > offs[:-1]
    unv = np.flatnonzero(unvisited)
    if unv.shape[0] == 0:
        return 0, 0
    deg = offs[unv + 1] - offs[unv]
    total = int(deg.sum())
    probes = deg.copy()
    if total:
        csum = np.zeros(unv.shape[0] + 1, dtype=np.int64)
        np.cumsum(deg, out=csum[1:])
        row = np.repeat(np.arange(unv.shape[0], dtype=np.int64), deg)
        pos = np.arange(total, dtype=np.int64) - csum[row]
        hit = lv[cols[offs[unv][row] + pos]] == d
        hr, hp = row[hit], pos[hit]
        if hr.shape[0]:
            first = np.empty(hr.shape[0], dtype=bool)
            first[0] = True
            first[1:] = hr[1:] != hr[:-1]
            probes[hr[first]] = hp[first] + 1
    return int(probes.sum()), int(unv.shape[0])


def ranked_head(offs, cols, v: int):
    """The head of v as the library's single-source workspace builds it: the
    four neighbours of largest degree among the first 256 arcs, an earlier
    arc first among equal degrees."""
    deg = np.diff(np.asarray(offs, dtype=np.int64))
    row = np.asarray(cols[offs[v]:offs[v] + min(256, int(deg[v]))], dtype=np.int64)
    order = sorted(range(row.shape[0]), key=lambda e: (-int(deg[row[e]]), e))
    return [int(row[e]) for e in order[:4]]


def head_probes_reference(offs, cols, level, d: int, ranked: bool):
    """(probes, row reads) of a bottom-up level d starting from the head
    (ranked, or the row's first four arcs), by walking every unvisited
    vertex in Python (slow; the check of ``Counts``)."""
    offs = np.asarray(offs, dtype=np.int64)
    lv = np.asarray(level)
    r0 = 0 if ranked else 4
    probes = rows = 0
    for v in np.flatnonzero(((lv == -1) | (lv > d)) & (offs[1:] > offs[:-1])):
        deg = int(offs[v + 1] - offs[v])
        h = min(4, deg)
        head = ranked_head(offs, cols, int(v)) if ranked else [int(u) for u in cols[offs[v]:offs[v] + h]]
        if any(lv[u] == d for u in head):
            probes += h
            continue
        nb = lv[cols[offs[v]:offs[v + 1]]]
        hits = np.flatnonzero(nb == d)
        if deg >= 4:
            rows += 1
            probes += h + (int(hits[0]) + 1 if hits.shape[0] else deg) - r0
        else:
            probes += h
    return probes, rows
