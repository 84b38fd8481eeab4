"""Invariant checker: accepts valid BFS output, rejects planted mistakes.

Mistakes are planted in copies of the oracle's output on the CPU.
"""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1708_01159_amd import graphgen as gg


@pytest.fixture(scope="module")
def case():
    g = gg.rmat(10, 16, seed=1)
    s = int(gg.pick_sources(g, 1, 101)[0])
    lv, par, _, _ = oracle.bfs(g.offs, g.cols, s)
    comp = checks.components(g.n, g.offs, g.cols)
    return g, s, lv, par, comp


def test_accepts_oracle(case):
    g, s, lv, par, comp = case
    checks.check_bfs(g.offs, g.cols, s, lv, par, comp)


def _reject(g, s, lv, par, comp):
    with pytest.raises(checks.InvariantError):
        checks.check_bfs(g.offs, g.cols, s, lv, par, comp)


def test_rejects_off_by_one_level(case):
    g, s, lv, par, comp = case
    bad = lv.copy()
    v = int(np.flatnonzero(lv == lv.max())[0])
    bad[v] += 1
    _reject(g, s, bad, par, comp)
    bad = lv.copy()
    v = int(np.flatnonzero(lv == 2)[0])
    bad[v] = 1  # neighbour chain still fine but parent no longer one level up
    _reject(g, s, bad, par, comp)


def test_rejects_bad_source(case):
    g, s, lv, par, comp = case
    bad = lv.copy()
    bad[s] = 1
    _reject(g, s, bad, par, comp)
    badp = par.copy()
    badp[s] = -1
    _reject(g, s, lv, badp, comp)


def test_rejects_non_neighbour_parent(case):
    g, s, lv, par, comp = case
    v = int(np.flatnonzero(lv == 3)[0])
    nbrs = set(g.cols[g.offs[v]:g.offs[v + 1]].tolist())
    cand = [u for u in np.flatnonzero(lv == 2) if u not in nbrs]
    badp = par.copy()
    badp[v] = int(cand[0])
    _reject(g, s, lv, badp, comp)


def test_rejects_same_level_parent(case):
    g, s, lv, par, comp = case
    rows = np.repeat(np.arange(g.n), g.degrees())
    same = np.flatnonzero((lv[rows] == lv[g.cols]) & (lv[rows] > 0))
    e = int(same[0])
    badp = par.copy()
    badp[rows[e]] = g.cols[e]
    _reject(g, s, lv, badp, comp)


def test_rejects_unreached_mismatch(case):
    g, s, lv, par, comp = case
    unreached = np.flatnonzero(lv < 0)
    assert unreached.shape[0] > 0
    v = int(unreached[0])
    bad = lv.copy()
    bad[v] = 1
    badp = par.copy()
    badp[v] = s
    _reject(g, s, bad, badp, comp)
    # parent set on an unreached vertex (I4)
    badp = par.copy()
    badp[v] = s
    _reject(g, s, lv, badp, comp)
    # a reached vertex dropped (I2/I5)
    bad = lv.copy()
    badp = par.copy()
    w = int(np.flatnonzero(lv == lv.max())[0])
    bad[w] = -1
    badp[w] = -1
    _reject(g, s, bad, badp, comp)


def test_union_find_matches_scipy():
    g = gg.erdos_renyi(3000, 1800, seed=9)
    a = checks.components_union_find(g.n, g.offs, g.cols)
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    _, b = connected_components(sp.csr_matrix((np.ones(g.nnz), g.cols, g.offs), shape=(g.n, g.n)),
                                directed=False)
    # same partition: a bijection between labels
    pairs = set(zip(a.tolist(), b.tolist()))
    assert len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


def test_is_symmetric():
    g = gg.rmat(8, 8, seed=1)
    assert checks.is_symmetric(g.offs, g.cols)
    offs = np.array([0, 1, 1], dtype=np.int64)
    cols = np.array([1], dtype=np.int32)
    assert not checks.is_symmetric(offs, cols)


def _directed_graph():
    # a random directed graph with cycles, one-way and reciprocated arcs
    rng = np.random.default_rng(9)
    n, m = 300, 900
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    return gg.from_edges(n, src, dst, symmetrize=False, name="dir300")


def test_directed_invariants_accept_the_oracle():
    g = _directed_graph()
    assert not checks.is_symmetric(g.offs, g.cols)
    for s in gg.pick_sources(g, 5, 3):
        lv, pa, _, _ = oracle.bfs(g.offs, g.cols, int(s))
        checks.check_bfs_directed(g.offs, g.cols, int(s), lv, pa)
        # and the oracle equals scipy's directed shortest paths
        import scipy.sparse as sp
        from scipy.sparse.csgraph import shortest_path

        a = sp.csr_matrix((np.ones(g.nnz), g.cols, g.offs), shape=(g.n, g.n))
        d = shortest_path(a, directed=True, unweighted=True, indices=int(s))
        assert np.array_equal(np.where(np.isinf(d), -1, d).astype(np.int64), lv)


def test_directed_invariants_reject_planted_mistakes():
    g = _directed_graph()
    s = int(gg.pick_sources(g, 1, 4)[0])
    lv, pa, _, _ = oracle.bfs(g.offs, g.cols, s)
    deep = int(np.flatnonzero(lv == lv.max())[0])
    bad = lv.copy()
    bad[deep] += 1  # one level too deep: its parent's arc spans two levels
    with pytest.raises(checks.InvariantError):
        checks.check_bfs_directed(g.offs, g.cols, s, bad, pa)
    # a parent one level up that has no arc into the vertex (only a reverse one or none)
    rows = np.repeat(np.arange(g.n), g.degrees())
    v = deep
    ins = set(rows[g.cols == v].tolist())
    cands = [u for u in np.flatnonzero(lv == lv[v] - 1).tolist() if u not in ins]
    if cands:
        p2 = pa.copy()
        p2[v] = cands[0]
        with pytest.raises(checks.InvariantError):
            checks.check_bfs_directed(g.offs, g.cols, s, lv, p2)
    # an unreachable vertex reported reached
    un = np.flatnonzero(lv < 0)
    if un.size:
        l3, p3 = lv.copy(), pa.copy()
        l3[un[0]], p3[un[0]] = lv.max() + 1, deep
        with pytest.raises(checks.InvariantError):
            checks.check_bfs_directed(g.offs, g.cols, s, l3, p3)
    # the symmetric checker's I2 would reject a correct directed result (an
    # arc pointing back up more than one level is fine when directed)
    span = (lv[rows] >= 0) & (lv[g.cols] >= 0) & (lv[rows] - lv[g.cols] > 1)
    assert span.any()
