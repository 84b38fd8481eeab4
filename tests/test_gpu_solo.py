"""Single-workgroup multi-level launches (small frontiers): results equal the
oracle and the same search with those launches off -- levels bit-exact,
parents valid (canonical parents equal), every trace row equal except the
flag that marks the levels such a launch ran -- across the ways such a
launch starts and stops: from the first level, after and before full-grid
levels (the frontier bitmaps are rebuilt when it stops), at its level cap,
at a level whose arcs are too many for one workgroup, with rows long enough
to be spread over the workgroup, on directed graphs and under every policy."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw, trees

pytestmark = pytest.mark.gpu

SOLO = 4  # trace flag of a level run by a single-workgroup launch


def _path(n):
    return gg.from_edges(n, list(range(n - 1)), list(range(1, n)), name="path%d" % n)


def _caterpillar(spine, legs):
    """A path of `spine` vertices, each with `legs` leaves: rows of legs + 2
    arcs, longer than a thread walks alone."""
    src, dst = list(range(spine - 1)), list(range(1, spine))
    leaf = spine
    for v in range(spine):
        for _ in range(legs):
            src.append(v)
            dst.append(leaf)
            leaf += 1
    return gg.from_edges(leaf, src, dst, name="caterpillar")


def _path_then_hub(path_len, leaves):
    """A path whose far end is a hub with `leaves` leaves: the tail rule lets
    small levels run in one workgroup until the hub's level, whose arcs are
    too many for it."""
    n = path_len + 1 + leaves
    src = list(range(path_len - 1)) + [path_len - 1] + [path_len] * leaves
    dst = list(range(1, path_len)) + [path_len] + list(range(path_len + 1, n))
    return gg.from_edges(n, src, dst, name="path_hub")


CASES = {
    "grid_ragged": lambda: gg.grid(97, 83, 0.05, seed=51),
    "grid_full": lambda: gg.grid(200, 200, 0.0, seed=52),
    "path3000": lambda: _path(3000),
    "caterpillar": lambda: _caterpillar(400, 20),
    "path_hub": lambda: _path_then_hub(3000, 120000),
    "rmat14": lambda: gg.rmat(14, 16, seed=11),
    "er_sparse": lambda: gg.erdos_renyi(30011, 40000, seed=53),
}

_cache = {}


def case(name):
    if name not in _cache:
        g = CASES[name]()
        if name in ("path3000", "path_hub", "caterpillar"):
            srcs = np.array([0, 5], dtype=np.int32)
        else:
            srcs = gg.pick_sources(g, 3, 57)
        G = gsw.Graph.from_csr(g.offs, g.cols)
        refs = [oracle.bfs(g.offs, g.cols, int(s)) for s in srcs]
        _cache[name] = (g, G, srcs, refs)
    return _cache[name]


def _key(rows):
    return [(t.source_idx, t.level, t.kernel, t.flags & ~SOLO, t.n_frontier, t.discovered, t.n_next, t.e_frontier)
            for t in rows]


def _run_both(name, **kw):
    g, G, srcs, refs = case(name)
    lv1, pa1, tr1 = gsw.bfs(G, srcs, solo=True, count_arcs=True, canonical_parents=True, **kw)
    lv0, pa0, tr0 = gsw.bfs(G, srcs, solo=False, count_arcs=True, canonical_parents=True, **kw)
    assert np.array_equal(lv1, lv0)
    assert np.array_equal(pa1, pa0)
    assert _key(tr1) == _key(tr0)
    assert not any(t.flags & SOLO for t in tr0)
    for i, s in enumerate(srcs):
        ref_lv, _, hist, ehist = refs[i]
        assert np.array_equal(lv1[i], ref_lv), "levels differ for source %d" % s
        checks.check_bfs(g.offs, g.cols, int(s), lv1[i], pa1[i])
        rows = [t for t in tr1 if t.source_idx == i]
        assert [t.n_frontier for t in rows] == hist.tolist()
        assert [t.e_frontier for t in rows] == ehist.tolist()
    return tr1


@pytest.mark.parametrize("name", list(CASES))
def test_solo_tree_policy(name):
    tr = _run_both(name, policy="tree", tree=trees.load_default())
    if name in ("grid_ragged", "grid_full", "path3000"):  # the tree pushes on some of their small levels
        assert any(t.flags & SOLO for t in tr)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("base", [gsw.PUSH_VERTEX, gsw.PUSH_WAVE4, gsw.PUSH_WAVE32, gsw.PUSH_EDGE])
def test_solo_fixed_push_kernels(name, base):
    for variant in (gsw.COUNT_WORKGROUP, gsw.COUNT_WAVE, gsw.COUNT_THREAD):
        k = gsw.kernel_id(base, variant)
        tr = _run_both(name, policy="fixed", kernel=k)
        assert all(t.kernel == k for t in tr)
        if name in ("grid_full", "path3000"):
            # from the first level on; after each single-workgroup launch (at
            # most 32 levels) one full-grid launch follows
            assert tr[0].flags & SOLO
            assert sum(1 for t in tr if t.flags & SOLO) >= 0.9 * len(tr)


def test_solo_path_levels_past_the_cap():
    # 2999 levels from one end: about a hundred launches of at most 32 levels each
    tr = _run_both("path3000", policy="fixed", kernel=gsw.PUSH_VERTEX)
    assert len([t for t in tr if t.source_idx == 0]) == 3000


def test_solo_hub_level_goes_back_to_the_grid():
    g, G, srcs, refs = case("path_hub")
    tr = _run_both("path_hub", policy="fixed", kernel=gsw.PUSH_EDGE)
    for i in range(len(srcs)):
        rows = [t for t in tr if t.source_idx == i]
        hub = [t for t in rows if t.e_frontier > 65536]
        assert hub and not any(t.flags & SOLO for t in hub)
        # the tail rule took over once 1% of the graph was reached
        assert any(t.flags & SOLO for t in rows)


@pytest.mark.parametrize("name", ["grid_ragged", "caterpillar", "rmat14", "er_sparse"])
def test_solo_stops_before_pull_and_starts_again(name):
    """Schedules that switch between push and pull: every stop rebuilds the
    frontier bitmaps the pull level reads."""
    g, G, srcs, refs = case(name)
    depth = max(len(r[2]) for r in refs)
    rng = np.random.default_rng(7)
    push = [gsw.PUSH_VERTEX, gsw.PUSH_WAVE8, gsw.PUSH_EDGE, gsw.kernel_id(gsw.PUSH_VERTEX, gsw.COUNT_THREAD)]
    for trial in range(4):
        sched = [int(rng.choice(push)) if rng.random() < 0.7 else
                 int(rng.choice([gsw.PULL_BITMAP, gsw.VERTEX_SCAN, gsw.REV_EDGE_SCAN])) for _ in range(depth)]
        tr = _run_both(name, policy="schedule", schedule=np.array(sched, dtype=np.int32))
        for t in tr:
            assert t.kernel == sched[min(t.level, depth - 1)]


def test_solo_directed_graph():
    a = gg.grid(61, 67, 0.0, seed=55)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = np.random.default_rng(5).random(a.nnz) < 0.75
    g = gg.from_edges(a.n, rows[keep], a.cols[keep], symmetrize=False, name="grid_dir")
    G = gsw.Graph.from_csr(g.offs, g.cols)
    srcs = gg.pick_sources(g, 3, 59)
    for kernel in (gsw.PUSH_VERTEX, gsw.PUSH_EDGE):
        lv1, pa1, tr1 = gsw.bfs(G, srcs, policy="fixed", kernel=kernel, solo=True, canonical_parents=True)
        lv0, pa0, tr0 = gsw.bfs(G, srcs, policy="fixed", kernel=kernel, solo=False, canonical_parents=True)
        assert np.array_equal(lv1, lv0) and np.array_equal(pa1, pa0)
        assert any(t.flags & SOLO for t in tr1)
        for i, s in enumerate(srcs):
            assert np.array_equal(lv1[i], oracle.levels(g.offs, g.cols, int(s)))
            checks.check_bfs_directed(g.offs, g.cols, int(s), lv1[i], pa1[i])
    G.close()


def test_solo_timed_levels_and_device_outputs():
    import torch

    g, G, srcs, refs = case("grid_ragged")
    lv = torch.full((len(srcs), g.n), 9, dtype=torch.int32, device="cuda")
    pa = torch.full((len(srcs), g.n), 9, dtype=torch.int32, device="cuda")
    _, _, tr = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PUSH_VERTEX, time_levels=True, device=True,
                       out=(lv, pa))
    torch.cuda.synchronize()
    solo = [t for t in tr if t.flags & SOLO]
    assert solo and all(t.ms > 0.0 for t in solo)
    for i, s in enumerate(srcs):
        assert np.array_equal(lv[i].cpu().numpy(), refs[i][0])
    # per-launch events cannot time levels that share a launch: none run there
    _, _, tr = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PUSH_VERTEX, time_levels=2)
    assert not any(t.flags & SOLO for t in tr) and all(t.ms > 0.0 for t in tr)
