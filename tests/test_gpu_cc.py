"""Weakly connected components on the GPU (gsw_cc) against the oracle's
disjoint-set forest: labels (the smallest id of each component) bit-exact and
the component count, under every policy, with and without the BFS phase, on
graphs with one giant component, many small ones, long paths, isolated
vertices, repeated arcs and loops, directed arcs, and at full size."""
import numpy as np
import pytest

import oracle
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw, trees

pytestmark = pytest.mark.gpu


def _paths(lengths):
    src, dst, base = [], [], 0
    for m in lengths:
        src += list(range(base, base + m - 1))
        dst += list(range(base + 1, base + m))
        base += m
    return gg.from_edges(base + 5, src, dst, name="paths")  # plus 5 isolated vertices


def _two_grids():
    a = gg.grid(60, 60, 0.0, seed=31)
    rows = np.repeat(np.arange(a.n), a.degrees())
    src = np.concatenate([rows, rows + a.n])
    dst = np.concatenate([a.cols, a.cols + a.n])
    return gg.from_edges(2 * a.n, src, dst, name="two_grids")


def _multi():
    rng = np.random.default_rng(33)
    src = rng.integers(0, 3000, 5000)
    dst = rng.integers(0, 3000, 5000)
    src = np.concatenate([src, src[:500], np.arange(100)])  # repeats and loops
    dst = np.concatenate([dst, dst[:500], np.arange(100)])
    return gg.from_edges(3000, src, dst, drop_loops=False, dedup=False, name="multi")


def _directed():
    a = gg.grid(70, 50, 0.0, seed=34)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = np.random.default_rng(35).random(a.nnz) < 0.35
    return gg.from_edges(a.n, rows[keep], a.cols[keep], symmetrize=False, name="grid_dir")


CASES = {
    "rmat14": lambda: gg.rmat(14, 16, seed=21),
    "grid_holes": lambda: gg.grid(120, 90, 0.45, seed=22),
    "er_sparse": lambda: gg.erdos_renyi(20011, 12000, seed=23),
    "paths": lambda: _paths([1, 2, 3, 17, 64, 65, 3000, 129]),
    "two_grids": _two_grids,
    "multi": _multi,
    "directed": _directed,
}

_cache = {}


def case(name):
    if name not in _cache:
        g = CASES[name]()
        G = gsw.Graph.from_csr(g.offs, g.cols)
        _cache[name] = (g, G, oracle.components(g.offs, g.cols))
    return _cache[name]


def _check(name, **kw):
    g, G, (want, count) = case(name)
    lab, nc, tr = gsw.components(G, **kw)
    assert np.array_equal(lab, want), "labels differ on %s %s" % (name, kw)
    assert nc == count
    return g, G, tr


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("policy", ["switch", "push", "pull"])
@pytest.mark.parametrize("bfs_first", [True, False])
def test_components_equal_oracle(name, policy, bfs_first):
    g, G, tr = _check(name, policy=policy, bfs_first=bfs_first, tree=trees.load_default())
    phase1 = bfs_first and G.symmetric and g.nnz > 0
    assert (tr[0]["kernel"] == "bfs") == phase1
    it = tr[1:] if phase1 else tr
    if g.nnz > 0 and it:
        assert it[-1]["changed"] == 0  # the last iteration changed nothing
        assert all(r["changed"] > 0 for r in it[:-1])
    if policy != "switch":
        assert all(r["kernel"] == policy for r in it)


def test_phase1_row_reaches_the_largest_degree_component():
    g, G, (want, _) = case("rmat14")
    _, _, tr = _check("rmat14", tree=trees.load_default())
    seed = int(np.argmax(g.degrees()))
    assert tr[0]["kernel"] == "bfs" and tr[0]["changed"] == int((want == want[seed]).sum())


def test_switch_rule():
    """The switch policy pulls exactly when the active arcs exceed pull_above
    of the arcs left to propagation (the first iteration's active set is all
    of them)."""
    for pull_above in (0.0, 0.05, 0.5, 2.0):
        g, G, tr = _check("grid_holes", policy="switch", bfs_first=True, pull_above=pull_above)
        it = tr[1:]
        e_rest = it[0]["e_active"]
        for r in it:
            want = "pull" if r["e_active"] > pull_above * e_rest else "push"
            assert r["kernel"] == want, (pull_above, r)


def test_no_arcs_and_single_vertex():
    for n in (1, 1000):
        G = gsw.Graph.from_csr(np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32))
        for policy in ("switch", "push", "pull"):
            lab, nc, tr = gsw.components(G, policy=policy)
            assert np.array_equal(lab, np.arange(n)) and nc == n and tr == []
        G.close()


def test_device_output_and_repeat_calls():
    import torch

    g, G, (want, count) = case("er_sparse")
    out = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
    for _ in range(3):  # the graph's working memory is reused
        lab, nc, _ = gsw.components(G, device=True, out=out, tree=trees.load_default())
        torch.cuda.synchronize()
        assert nc == count and np.array_equal(out.cpu().numpy(), want)
    with pytest.raises(ValueError):
        gsw.components(G, device=True, out=torch.empty(g.n - 1, dtype=torch.int32, device="cuda"))
    host = np.full(g.n, 7, dtype=np.int32)
    lab, nc, _ = gsw.components(G, out=host, tree=trees.load_default())
    assert lab is host and nc == count and np.array_equal(host, want)


def test_full_size_rmat22():
    g = gg.workload("rmat22")
    want, count = oracle.components(g.offs, g.cols)
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    for policy in ("switch", "pull"):
        lab, nc, tr = gsw.components(G, policy=policy, tree=trees.load_default())
        assert nc == count and np.array_equal(lab, want), policy
    G.close()
