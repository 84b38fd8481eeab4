"""Graph500-style BFS invariants and connected components (test infrastructure).

Written independently of the FIFO oracle.  For a source s, levels L and
parents P over an undirected CSR graph:

  I1  L[s] == 0 and P[s] == s;
  I2  every arc (u, v) with L[u] >= 0 has L[v] >= 0 and |L[u] - L[v]| <= 1;
  I3  every reached v != s has P[v] adjacent to v with L[P[v]] == L[v] - 1;
  I4  L[v] == -1 exactly when P[v] == -1;
  I5  the reached set equals the connected component of s.

I1 + I2 + I3 + I5 force L to be the hop distance from s: the parent chain is
a path of length L[v] (so distance <= L[v]), and along a shortest path I2 lets
L grow by at most one per edge (so L[v] <= distance).  Parents are not unique;
these checks are what a parent array must pass.
"""
from __future__ import annotations

import numpy as np


class InvariantError(AssertionError):
    pass


def _rows(offs: np.ndarray) -> np.ndarray:
    n = offs.shape[0] - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(offs))


def components_union_find(n: int, offs, cols) -> np.ndarray:
    """Component label per vertex by union-find with path halving (pure
    Python; for small graphs).  Labels are the smallest vertex id of each
    component."""
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u in range(n):
        for e in range(int(offs[u]), int(offs[u + 1])):
            a, b = find(u), find(int(cols[e]))
            if a != b:
                if a < b:
                    parent[b] = a
                else:
                    parent[a] = b
    return np.array([find(v) for v in range(n)], dtype=np.int64)


def components(n: int, offs, cols) -> np.ndarray:
    """Component labels; union-find for small graphs, scipy's routine above
    that (a library primitive, not a BFS)."""
    offs = np.asarray(offs, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if n <= 4096:
        return components_union_find(n, offs, cols)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.csr_matrix((np.ones(cols.shape[0], dtype=np.int8), cols, offs), shape=(n, n))
    _, lab = connected_components(a, directed=False)
    return lab.astype(np.int64)


def check_bfs(offs, cols, source: int, level, parent=None, comp=None) -> None:
    """Raise InvariantError unless (level, parent) is a valid BFS from source."""
    offs = np.asarray(offs, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    level = np.asarray(level, dtype=np.int64)
    n = offs.shape[0] - 1
    s = int(source)
    if level.shape != (n,):
        raise InvariantError("level has shape %r, expected (%d,)" % (level.shape, n))
    # I1
    if level[s] != 0:
        raise InvariantError("I1: level[source]=%d" % level[s])
    rows = _rows(offs)
    # I2
    lu = level[rows]
    lv = level[cols]
    live = lu >= 0
    if np.any(lv[live] < 0):
        e = int(np.flatnonzero(live & (lv < 0))[0])
        raise InvariantError("I2: arc (%d,%d) leaves the reached set" % (rows[e], cols[e]))
    if np.any(np.abs(lu[live] - lv[live]) > 1):
        e = int(np.flatnonzero(live & (np.abs(lu - lv) > 1))[0])
        raise InvariantError("I2: arc (%d,%d) spans levels %d,%d" % (rows[e], cols[e], lu[e], lv[e]))
    if np.any(level < -1):
        raise InvariantError("level below -1")
    if parent is not None:
        parent = np.asarray(parent, dtype=np.int64)
        if parent[s] != s:
            raise InvariantError("I1: parent[source]=%d" % parent[s])
        # I4
        if np.any((level == -1) != (parent == -1)):
            v = int(np.flatnonzero((level == -1) != (parent == -1))[0])
            raise InvariantError("I4: vertex %d has level %d parent %d" % (v, level[v], parent[v]))
        # I3
        vs = np.flatnonzero(level > 0)
        ps = parent[vs]
        if np.any((ps < 0) | (ps >= n)):
            raise InvariantError("I3: parent out of range")
        if np.any(level[ps] != level[vs] - 1):
            i = int(np.flatnonzero(level[ps] != level[vs] - 1)[0])
            raise InvariantError("I3: parent %d of %d is not one level up" % (ps[i], vs[i]))
        key = rows * n + cols
        if key.shape[0] > 1 and not np.all(key[1:] >= key[:-1]):
            key = np.sort(key)
        want = vs.astype(np.int64) * n + ps
        pos = np.searchsorted(key, want)
        pos = np.minimum(pos, max(key.shape[0] - 1, 0))
        if key.shape[0] == 0 and vs.shape[0] > 0:
            raise InvariantError("I3: parent on an edgeless graph")
        bad = key[pos] != want if key.shape[0] else np.zeros(0, dtype=bool)
        if np.any(bad):
            i = int(np.flatnonzero(bad)[0])
            raise InvariantError("I3: parent %d is not adjacent to %d" % (ps[i], vs[i]))
    # I5
    if comp is None:
        comp = components(n, offs, cols)
    reached = level >= 0
    incomp = comp == comp[s]
    if np.any(reached != incomp):
        v = int(np.flatnonzero(reached != incomp)[0])
        raise InvariantError("I5: vertex %d reached=%s in-component=%s" % (v, reached[v], incomp[v]))


def reachable(offs, cols, source: int) -> np.ndarray:
    """Vertices reachable from ``source`` along arcs (scipy's traversal, a
    library routine independent of the FIFO oracle)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order

    offs = np.asarray(offs, dtype=np.int64)
    n = offs.shape[0] - 1
    a = sp.csr_matrix((np.ones(len(cols), dtype=np.int8), np.asarray(cols, dtype=np.int64), offs), shape=(n, n))
    order = breadth_first_order(a, int(source), directed=True, return_predecessors=False)
    out = np.zeros(n, dtype=bool)
    out[order] = True
    return out


def check_bfs_directed(offs, cols, source: int, level, parent=None) -> None:
    """The invariants for a directed graph (row u lists the arcs u -> v):

      D1  L[s] == 0 and P[s] == s;
      D2  every arc (u, v) with L[u] >= 0 has L[v] >= 0 and L[v] <= L[u] + 1;
      D3  every reached v != s has an arc P[v] -> v with L[P[v]] == L[v] - 1;
      D4  L[v] == -1 exactly when P[v] == -1;
      D5  the reached set equals the set reachable from s.

    D3 gives a path of length L[v] (distance <= L[v]); along a shortest path
    D2 raises L by at most one per arc (L[v] <= distance)."""
    offs = np.asarray(offs, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    level = np.asarray(level, dtype=np.int64)
    n = offs.shape[0] - 1
    s = int(source)
    if level[s] != 0:
        raise InvariantError("D1: level[source]=%d" % level[s])
    rows = _rows(offs)
    lu, lv = level[rows], level[cols]
    live = lu >= 0
    if np.any(lv[live] < 0) or np.any(lv[live] > lu[live] + 1):
        e = int(np.flatnonzero(live & ((lv < 0) | (lv > lu + 1)))[0])
        raise InvariantError("D2: arc (%d,%d) has levels %d,%d" % (rows[e], cols[e], lu[e], lv[e]))
    if parent is not None:
        parent = np.asarray(parent, dtype=np.int64)
        if parent[s] != s:
            raise InvariantError("D1: parent[source]=%d" % parent[s])
        if np.any((level == -1) != (parent == -1)):
            raise InvariantError("D4: reached and parent disagree")
        vs = np.flatnonzero(level > 0)
        ps = parent[vs]
        if np.any((ps < 0) | (ps >= n)) or np.any(level[ps] != level[vs] - 1):
            raise InvariantError("D3: a parent is not one level up")
        arcs = set((rows * n + cols).tolist())
        for v, p in zip(vs.tolist(), ps.tolist()):
            if p * n + v not in arcs:
                raise InvariantError("D3: no arc %d -> %d" % (p, v))
    if np.any((level >= 0) != reachable(offs, cols, s)):
        raise InvariantError("D5: reached set differs from the reachable set")


def is_symmetric(offs, cols) -> bool:
    offs = np.asarray(offs, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    n = offs.shape[0] - 1
    rows = _rows(offs)
    a = np.sort(rows * n + cols)
    b = np.sort(cols * n + rows)
    return bool(np.array_equal(a, b))
