"""Algorithmic HBM bytes of one BFS level, per kernel family, and TEPS counts.

Measurement arithmetic for the roofline: what each expansion kernel must move
at level d, counted at the granularity it accesses (4-byte ids and levels,
8-byte offsets, 64-bit bitmap words).  Computed exactly on the host from a
level array (the GPU's own output) and the sorted CSR.

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
  pull_bitmap    + nw*8 (visited words) + sum over unvisited v of
                 (16 row offsets + p_v*(4 column + 8 frontier word))
                 + 16 per word holding a discovery (visited and next words),
                 where p_v counts the neighbours read up to the first one in
                 the frontier (all of them when none is).  On a symmetric
                 graph degree-0 vertices start visited (the search marks them
                 at init), so they cost only their visited bit.
"""
from __future__ import annotations

import numpy as np

PUSH_FAMILY = (0, 1, 2, 3, 4, 5)
PUSH_EDGE, PULL, VERTEX_SCAN, EDGE_SCAN = 6, 7, 8, 9


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


def pull_probes(offs, cols, level, d: int, skip_isolated: bool = True):
    """(sum of p_v, unvisited count, words with a discovery) for a pull at
    level d; degree-0 vertices are left out when ``skip_isolated``."""
    offs = np.asarray(offs, dtype=np.int64)
    lv = np.asarray(level)
    n = lv.shape[0]
    unvisited = (lv == -1) | (lv > d)
    if skip_isolated:
        unvisited &= offs[1:] > offs[:-1]
    unv = np.flatnonzero(unvisited)
    if unv.shape[0] == 0:
        return 0, 0, 0
    deg = offs[unv + 1] - offs[unv]
    total = int(deg.sum())
    probes = deg.copy()
    if total:
        csum = np.zeros(unv.shape[0] + 1, dtype=np.int64)
        np.cumsum(deg, out=csum[1:])
        row = np.repeat(np.arange(unv.shape[0], dtype=np.int64), deg)
        pos = np.arange(total, dtype=np.int64) - csum[row]
        hit = lv[cols[offs[unv][row] + pos]] == d
        hr = row[hit]
        hp = pos[hit]
        if hr.shape[0]:
            first = np.empty(hr.shape[0], dtype=bool)
            first[0] = True
            first[1:] = hr[1:] != hr[:-1]
            probes[hr[first]] = hp[first] + 1
    found_words = np.unique(np.flatnonzero(lv == d + 1) >> 6).shape[0]
    return int(probes.sum()), int(unv.shape[0]), int(found_words)


def level_bytes(kernel: int, offs, cols, level, d: int, nf=None, ef=None, skip_isolated: bool = True) -> int:
    """Algorithmic bytes of running ``kernel`` at level d (see module doc);
    ``skip_isolated``: the graph is symmetric, degree-0 vertices start visited."""
    offs = np.asarray(offs, dtype=np.int64)
    lv = np.asarray(level)
    n = lv.shape[0]
    nnz = int(offs[-1])
    nw = (n + 63) // 64
    if nf is None or ef is None:
        nf, ef = level_sizes(offs, lv)
    n_f = int(nf[d]) if d < nf.shape[0] else 0
    e_f = int(ef[d]) if d < ef.shape[0] else 0
    n_x = int(nf[d + 1]) if d + 1 < nf.shape[0] else 0
    b = nw * 8 + n_x * 12
    if kernel == PULL:
        p, nu, words = pull_probes(offs, cols, lv, d, skip_isolated)
        return b + nw * 8 + nu * 16 + p * 12 + words * 16
    b += e_f * 12 + n_x * 8
    if kernel in PUSH_FAMILY:
        return b + n_f * 20
    if kernel == PUSH_EDGE:
        return b + n_f * (20 + 16 + 20)
    if kernel == VERTEX_SCAN:
        return b + n * 4 + n_f * 16
    if kernel == EDGE_SCAN:
        return b + nnz * 4 + n * 4
    raise ValueError("unknown kernel %r" % kernel)
