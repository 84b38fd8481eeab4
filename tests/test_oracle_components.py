"""Pins of the weakly-connected-components oracle (``oracle.components``):
closed forms, brute-force reachability on tiny graphs (directed arcs taken
both ways), scipy's connected-components routine on larger ones, and planted
mistakes in the C source that these pins must catch."""
import os
import re

import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1708_01159_amd import graphgen as gg

from test_oracle_bfs import csr_numpy


def brute_labels(n, offs, cols):
    """Smallest id of every vertex's weak component by boolean closure of the
    symmetrised adjacency (Floyd-Warshall on reachability)."""
    r = np.eye(n, dtype=bool)
    for u in range(n):
        for e in range(offs[u], offs[u + 1]):
            r[u, cols[e]] = r[cols[e], u] = True
    for k in range(n):
        r = r | (r[:, k:k + 1] & r[k:k + 1, :])
    return np.array([int(np.flatnonzero(r[:, v])[0]) for v in range(n)], dtype=np.int32)


def random_directed(rng, n):
    p = rng.choice([0.01, 0.03, 0.08, 0.2])
    pairs = [(u, v) for u in range(n) for v in range(n) if u != v and rng.random() < p]
    for _ in range(rng.integers(0, 3)):  # loops and a repeat
        u = int(rng.integers(0, n))
        pairs.append((u, u))
    if pairs and rng.random() < 0.5:
        pairs.append(pairs[0])
    return pairs


def test_closed_forms():
    # a path, in either direction of its arcs: one component
    for pairs, sym in (([(i, i + 1) for i in range(9)], True), ([(i, i + 1) for i in range(9)], False),
                       ([(i + 1, i) for i in range(9)], False)):
        offs, cols = csr_numpy(10, pairs, symmetrize=sym)
        lab, c = oracle.components(offs, cols)
        assert c == 1 and not lab.any()
    # no arcs: every vertex alone
    lab, c = oracle.components(np.zeros(8, dtype=np.int64), np.zeros(0, dtype=np.int32))
    assert c == 7 and np.array_equal(lab, np.arange(7))
    # k disjoint cliques of s vertices, listed from the highest block down
    k, s = 5, 4
    pairs = [(b * s + i, b * s + j) for b in reversed(range(k)) for i in range(s) for j in range(i + 1, s)]
    offs, cols = csr_numpy(k * s, pairs)
    lab, c = oracle.components(offs, cols)
    assert c == k and np.array_equal(lab, np.repeat(np.arange(k) * s, s))
    # a star whose centre is the largest id, plus isolated vertices around it
    n = 12
    pairs = [(n - 2, v) for v in range(2, n - 2)]
    offs, cols = csr_numpy(n, pairs)
    lab, c = oracle.components(offs, cols)
    want = np.arange(n, dtype=np.int32)
    want[2:n - 1] = 2
    assert c == 4 and np.array_equal(lab, want)  # {0}, {1}, {2..10}, {11}


def test_matches_brute_force_reachability():
    rng = np.random.default_rng(3)
    for trial in range(80):
        n = int(rng.integers(1, 30))
        directed = trial % 2 == 1
        pairs = random_directed(rng, n) if directed else [
            (u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.08]
        offs, cols = csr_numpy(n, pairs, symmetrize=not directed)
        want = brute_labels(n, offs, cols)
        lab, c = oracle.components(offs, cols)
        assert np.array_equal(lab, want), (trial, n)
        assert c == len(np.unique(want))


def _canonical(lab):
    """Relabel arbitrary component ids by each component's smallest vertex."""
    first = {}
    for v, x in enumerate(lab.tolist()):
        first.setdefault(x, v)
    return np.array([first[x] for x in lab.tolist()], dtype=np.int32)


def test_matches_scipy_and_python_union_find():
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    graphs = [gg.rmat(12, 8, seed=4), gg.grid(60, 50, 0.3, seed=5), gg.erdos_renyi(3000, 1400, seed=6)]
    a = gg.grid(40, 40, 0.0, seed=7)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = np.random.default_rng(8).random(a.nnz) < 0.3
    graphs.append(gg.from_edges(a.n, rows[keep], a.cols[keep], symmetrize=False, name="grid_dir"))
    for g in graphs:
        lab, c = oracle.components(g.offs, g.cols)
        m = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.cols, g.offs), shape=(g.n, g.n))
        k, sl = connected_components(m, directed=True, connection="weak")
        assert c == k
        assert np.array_equal(lab, _canonical(sl)), g.name
        if g.n <= 4096 and checks.is_symmetric(g.offs, g.cols):
            assert np.array_equal(lab, checks.components_union_find(g.n, g.offs, g.cols))


# planted mistakes in the disjoint-set forest, each caught by a pin above
MUTANTS = {
    # links the smaller root under the larger: roots are no longer the smallest ids
    "link_order": (r"if \(a < b\)(\s+)up\[b\] = a;(\s+)else if \(b < a\)(\s+)up\[a\] = b;",
                   r"if (a < b)\1up[a] = b;\2else if (b < a)\3up[b] = a;"),
    # the last arc of every row is skipped
    "last_arc": (r"for \(int64_t e = offs\[u\]; e < offs\[u \+ 1\]; \+\+e\) \{\n      int32_t a",
                 "for (int64_t e = offs[u]; e + 1 < offs[u + 1]; ++e) {\n      int32_t a"),
    # labels read before the final finds: a vertex keeps an intermediate root
    "stale_label": (r"label\[v\] = cc_find\(up, \(int32_t\)v\);", "label[v] = up[v];"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_mutated_components(tmp_path, mutant):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "bfs_oracle.c")).read()
    a, b = MUTANTS[mutant]
    new = re.sub(a, b, src)
    assert new != src
    path = tmp_path / ("cc_%s.c" % mutant)
    path.write_text(new)
    lib = oracle.load(oracle.build(force=True, src=str(path), out=str(tmp_path / ("cc_%s.so" % mutant))))
    rng = np.random.default_rng(11)
    caught = False
    for trial in range(100):
        n = int(rng.integers(2, 30))
        offs, cols = csr_numpy(n, random_directed(rng, n), symmetrize=trial % 2 == 0)
        lab, _ = oracle.components(offs, cols, lib=lib)
        if not np.array_equal(lab, brute_labels(n, offs, cols)):
            caught = True
            break
    assert caught, "pin did not catch mutant %s" % mutant
