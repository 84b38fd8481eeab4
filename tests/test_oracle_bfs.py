"""Pins of the CPU BFS oracle against things other than itself.

* brute-force all-pairs shortest paths (Floyd-Warshall on unit weights) on
  hundreds of small random graphs, every source;
* scipy's and networkx's unweighted shortest paths on mid-size graphs;
* closed forms: paths, cycles, stars, complete and complete bipartite graphs,
  full grids (Manhattan distance), complete binary trees, hypercubes
  (binomial level sizes), disjoint unions, isolated sources;
* hand-solved fixtures under tests/golden/;
* mutated copies of the oracle source (LIFO order, a wrong increment, a
  dropped visited test) must fail these pins.
"""
import os
import re
import subprocess
from math import comb

import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1708_01159_amd import graphgen as gg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr_numpy(n, pairs, symmetrize=True):
    """Test-local CSR builder (no dedup, no loop removal, stable order)."""
    src = [u for u, v in pairs]
    dst = [v for u, v in pairs]
    if symmetrize:
        src, dst = src + dst, dst + src
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int32)
    order = np.argsort(src, kind="stable")
    offs = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offs, src + 1, 1)
    return np.ascontiguousarray(np.cumsum(offs)), np.ascontiguousarray(dst[order])


def floyd_warshall(n, offs, cols):
    inf = np.iinfo(np.int64).max // 4
    d = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for u in range(n):
        for e in range(offs[u], offs[u + 1]):
            if cols[e] != u:
                d[u, cols[e]] = 1
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return np.where(d >= inf, -1, d)


def random_small_graph(rng, n):
    p = rng.choice([0.02, 0.05, 0.1, 0.3, 0.7])
    pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    # a few loops and repeats: tolerated input, must not change distances
    for _ in range(rng.integers(0, 3)):
        u = int(rng.integers(0, n))
        pairs.append((u, u))
    if pairs and rng.random() < 0.5:
        pairs.append(pairs[0])
    return pairs


def test_oracle_matches_floyd_warshall_all_sources():
    rng = np.random.default_rng(12345)
    for trial in range(300):
        n = int(rng.integers(1, 65))
        offs, cols = csr_numpy(n, random_small_graph(rng, n))
        dist = floyd_warshall(n, offs, cols)
        for s in range(n):
            lv, par, hist, ehist = oracle.bfs(offs, cols, s)
            assert np.array_equal(lv, dist[s]), (trial, n, s)
            assert hist.sum() == (lv >= 0).sum()
            assert np.array_equal(hist, np.bincount(lv[lv >= 0], minlength=hist.shape[0]))


def test_oracle_matches_scipy_and_networkx():
    import networkx as nx
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    graphs = [gg.rmat(12, 8, seed=21), gg.erdos_renyi(10000, 12000, seed=22),
              gg.grid(60, 70, 0.2, seed=23), gg.chung_lu(5000, 2.1, 6.0, seed=24)]
    for g in graphs:
        a = sp.csr_matrix((np.ones(g.nnz), g.cols, g.offs), shape=(g.n, g.n))
        srcs = gg.pick_sources(g, 4, 99)
        d = shortest_path(a, directed=False, unweighted=True, indices=srcs)
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        rows = np.repeat(np.arange(g.n), g.degrees())
        G.add_edges_from(zip(rows.tolist(), g.cols.tolist()))
        for i, s in enumerate(srcs):
            lv = oracle.levels(g.offs, g.cols, int(s))
            want = np.where(np.isinf(d[i]), -1, d[i]).astype(np.int64)
            assert np.array_equal(lv, want), g.name
            nxd = nx.single_source_shortest_path_length(G, int(s))
            want2 = np.full(g.n, -1)
            for v, dv in nxd.items():
                want2[v] = dv
            assert np.array_equal(lv, want2), g.name


def _lv(n, pairs, s):
    offs, cols = csr_numpy(n, pairs)
    return oracle.bfs(offs, cols, s)


def test_closed_forms():
    n = 50
    path = [(i, i + 1) for i in range(n - 1)]
    for s in (0, 17, n - 1):
        assert np.array_equal(_lv(n, path, s)[0], np.abs(np.arange(n) - s))
    for n in (9, 10):
        cyc = [(i, (i + 1) % n) for i in range(n)]
        s = 3
        k = np.abs(np.arange(n) - s)
        assert np.array_equal(_lv(n, cyc, s)[0], np.minimum(k, n - k))
    star = [(0, i) for i in range(1, 12)]
    lv, par, hist, ehist = _lv(12, star, 0)
    assert lv.tolist() == [0] + [1] * 11 and hist.tolist() == [1, 11]
    assert ehist.tolist() == [11, 11]
    lv = _lv(12, star, 5)[0]
    assert lv[5] == 0 and lv[0] == 1 and all(lv[i] == 2 for i in range(1, 12) if i != 5)
    kn = [(u, v) for u in range(8) for v in range(u + 1, 8)]
    assert _lv(8, kn, 2)[0].tolist() == [1, 1, 0, 1, 1, 1, 1, 1]
    a, b = 3, 5
    kab = [(u, a + v) for u in range(a) for v in range(b)]
    lv = _lv(a + b, kab, 1)[0]
    assert lv.tolist() == [2, 0, 2] + [1] * b
    r, c = 7, 9
    grid = gg.grid(r, c, 0.0, seed=1)
    for s in (0, 31, r * c - 1):
        lv = oracle.levels(grid.offs, grid.cols, s)
        ii, jj = np.divmod(np.arange(r * c), c)
        si, sj = divmod(s, c)
        assert np.array_equal(lv, np.abs(ii - si) + np.abs(jj - sj))
    nt = 127
    tree = [(i, (i - 1) // 2) for i in range(1, nt)]
    lv = _lv(nt, tree, 0)[0]
    assert np.array_equal(lv, np.floor(np.log2(np.arange(nt) + 1)).astype(int))


def test_hypercube_binomial_levels():
    for k in (3, 6, 9):
        n = 1 << k
        pairs = [(v, v ^ (1 << b)) for v in range(n) for b in range(k) if v < v ^ (1 << b)]
        for s in (0, n - 1, 5 % n):
            lv, _, hist, _ = _lv(n, pairs, s)
            assert hist.tolist() == [comb(k, d) for d in range(k + 1)]
            assert np.array_equal(lv, [bin(v ^ s).count("1") for v in range(n)])


def test_disjoint_union_and_isolated_source():
    pairs = [(0, 1), (1, 2), (3, 4), (4, 5), (5, 3)]
    lv = _lv(7, pairs, 0)[0]
    assert lv.tolist() == [0, 1, 2, -1, -1, -1, -1]
    lv, par, hist, _ = _lv(7, pairs, 6)
    assert lv.tolist() == [-1] * 6 + [0] and par.tolist() == [-1] * 6 + [6] and hist.tolist() == [1]


def test_loops_and_repeats_do_not_change_levels():
    g = gg.rmat(9, 8, seed=5)
    rows = np.repeat(np.arange(g.n), g.degrees())
    pairs = list(zip(rows.tolist(), g.cols.tolist()))
    dirty = pairs + pairs[:100] + [(v, v) for v in range(0, g.n, 7)]
    offs, cols = csr_numpy(g.n, dirty, symmetrize=False)
    for s in gg.pick_sources(g, 5, 3):
        assert np.array_equal(oracle.levels(offs, cols, int(s)), oracle.levels(g.offs, g.cols, int(s)))


def read_golden(name):
    n, pairs, expect = None, [], {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line.startswith("n "):
                n = int(line.split()[1])
            elif line.startswith("e "):
                _, u, v = line.split()
                pairs.append((int(u), int(v)))
            elif line.startswith("levels "):
                head, vals = line[len("levels "):].split(":")
                expect[int(head)] = [int(x) for x in vals.split()]
    return n, pairs, expect


@pytest.mark.parametrize("name", ["petersen.txt", "house.txt"])
def test_golden_fixtures(name):
    n, pairs, expect = read_golden(name)
    for s, want in expect.items():
        assert _lv(n, pairs, s)[0].tolist() == want
    if name == "petersen.txt":
        for s in range(n):
            assert _lv(n, pairs, s)[2].tolist() == [1, 3, 6]


def test_oracle_parents_pass_invariants():
    for g in (gg.rmat(10, 16, seed=1), gg.grid(20, 30, 0.1, seed=2), gg.erdos_renyi(3000, 3000, seed=4)):
        comp = checks.components(g.n, g.offs, g.cols)
        for s in gg.pick_sources(g, 5, 7):
            lv, par, _, _ = oracle.bfs(g.offs, g.cols, int(s))
            checks.check_bfs(g.offs, g.cols, int(s), lv, par, comp)


MUTANTS = {
    # LIFO instead of FIFO: levels become DFS depths
    "lifo": (r"queue\[head\+\+\]", "queue[--tail]", r"while \(head < tail\)", "while (tail > 0)"),
    # wrong increment
    "plus2": (r"level\[u\] \+ 1", "level[u] + 2", None, None),
    # the visited test dropped: a vertex is relabelled by every later parent
    "novisit": (r"if \(level\[v\] == -1\)", "if (v != s)", None, None),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_mutated_oracle(tmp_path, mutant):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "bfs_oracle.c")).read()
    a, b, c, d = MUTANTS[mutant]
    new = re.sub(a, b, src)
    if c:
        new = re.sub(c, d, new)
    assert new != src
    if mutant == "novisit":
        # keep the mutant terminating: bound the queue by the arc count
        new = new.replace("malloc((size_t)n * sizeof(int32_t))",
                          "malloc((size_t)(n + offs[n] + 1) * sizeof(int32_t))")
        new = new.replace("queue[tail++] = v;", "if (tail < n + offs[n]) queue[tail++] = v;")
    path = tmp_path / ("m_%s.c" % mutant)
    path.write_text(new)
    lib = oracle.load(oracle.build(force=True, src=str(path), out=str(tmp_path / ("m_%s.so" % mutant))))
    rng = np.random.default_rng(7)
    caught = False
    for trial in range(60):
        n = int(rng.integers(4, 40))
        offs, cols = csr_numpy(n, random_small_graph(rng, n))
        dist = floyd_warshall(n, offs, cols)
        for s in range(n):
            # histograms off (NULL): a mutant may produce depths beyond n
            lv = np.empty(n, dtype=np.int32)
            par = np.empty(n, dtype=np.int32)
            lib.oracle_bfs(n, offs.ctypes.data, cols.ctypes.data, s, lv.ctypes.data,
                           par.ctypes.data, None, None)
            if not np.array_equal(lv, dist[s]):
                caught = True
                break
        if caught:
            break
    assert caught, "pin did not catch mutant %s" % mutant


def test_msbfs_oracle_cap():
    g = gg.rmat(10, 16, seed=1)
    srcs = gg.pick_sources(g, 8, 1)
    lv8, ok = oracle.msbfs_levels(g.offs, g.cols, srcs)
    assert ok and lv8.dtype == np.int8
    for i, s in enumerate(srcs):
        assert np.array_equal(lv8[i].astype(np.int32), oracle.levels(g.offs, g.cols, int(s)))
    n = 200
    offs, cols = csr_numpy(n, [(i, i + 1) for i in range(n - 1)])
    _, ok = oracle.msbfs_levels(offs, cols, [0])
    assert not ok
    _, ok = oracle.msbfs_levels(offs, cols, [100])  # ecc 100 <= 127
    assert ok


def test_component_edges():
    pairs = [(0, 1), (1, 2), (3, 4)]
    offs, cols = csr_numpy(5, pairs)
    lv = oracle.levels(offs, cols, 0)
    assert oracle.component_edges(offs, lv) == 2
