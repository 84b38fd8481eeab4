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
