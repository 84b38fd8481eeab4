"""GPU parity: every expansion kernel, random per-level schedules and the tree
policy against the CPU oracle.  Levels must match bit-exactly; parents are
not unique and must pass the Graph500-style invariants (or, in canonical
mode, equal the smallest neighbour one level up)."""
import numpy as np
import pytest

import oracle
from oracle import checks
from oracle import features as ofeat
from oracle import tree as otree
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw

pytestmark = pytest.mark.gpu

ALL_KERNELS = list(range(gsw.N_KERNELS))


def _path(n):
    return gg.from_edges(n, list(range(n - 1)), list(range(1, n)), name="path%d" % n)


def _star(n):
    return gg.from_edges(n, [0] * (n - 1), list(range(1, n)), name="star%d" % n)


def _disjoint():
    a = gg.rmat(8, 8, seed=31)
    # second copy shifted, plus 40 isolated vertices at the end
    rows = np.repeat(np.arange(a.n), a.degrees())
    src = np.concatenate([rows, rows + a.n])
    dst = np.concatenate([a.cols, a.cols + a.n])
    return gg.from_edges(2 * a.n + 40, src, dst, name="disjoint")


def _dirty():
    a = gg.rmat(9, 8, seed=32)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = rows < a.cols
    src = np.concatenate([rows[keep], rows[keep][:200], np.arange(0, a.n, 5)])
    dst = np.concatenate([a.cols[keep], a.cols[keep][:200], np.arange(0, a.n, 5)])
    return gg.from_edges(a.n, src, dst, symmetrize=True, drop_loops=False, dedup=False, name="dirty")


CASES = {
    "rmat10": lambda: gg.rmat(10, 16, seed=1),
    "rmat14": lambda: gg.rmat(14, 16, seed=11),
    "er_ragged": lambda: gg.erdos_renyi(100037, 300000, seed=12),
    "grid": lambda: gg.grid(37, 53, 0.05, seed=13),
    "chunglu": lambda: gg.chung_lu(20000, 2.1, 12.0, seed=14),
    "path": lambda: _path(300),
    "star": lambda: _star(5000),
    "disjoint": _disjoint,
    "dirty": _dirty,
    "single": lambda: gg.from_edges(1, [], [], name="single"),
}

_cache = {}


def case(name):
    if name not in _cache:
        g = CASES[name]()
        if name == "rmat10":
            srcs = gg.pick_sources(g, 1, 101)
        elif name == "single":
            srcs = np.array([0], dtype=np.int32)
        elif name == "disjoint":
            srcs = np.array([0, g.n // 2 - 20 + 3, g.n - 1], dtype=np.int32)  # incl. isolated
        elif name == "star":
            srcs = np.array([0, 17], dtype=np.int32)
        else:
            srcs = gg.pick_sources(g, 2, 7)
        G = gsw.Graph.from_csr(g.offs, g.cols)
        refs = [oracle.bfs(g.offs, g.cols, int(s)) for s in srcs]
        comp = checks.components(g.n, g.offs, g.cols)
        _cache[name] = (g, G, srcs, refs, comp)
    return _cache[name]


def _check_result(g, srcs, refs, comp, lv, pa, trace, arcs=False):
    """Levels bit-exact, parents valid, and the trace's per-level counts equal
    the oracle's histograms: n_f, n_next, discovered and -- when the run
    counted arcs -- e_f (the degree sum of each depth), else -1."""
    for i, s in enumerate(srcs):
        ref_lv, _, hist, ehist = refs[i]
        assert np.array_equal(lv[i], ref_lv), "levels differ for source %d" % s
        checks.check_bfs(g.offs, g.cols, int(s), lv[i], pa[i], comp)
        rows = [t for t in trace if t.source_idx == i]
        assert [t.level for t in rows] == list(range(len(hist)))
        assert [t.n_frontier for t in rows] == hist.tolist()
        assert [t.n_next for t in rows] == hist[1:].tolist() + [0]
        assert [t.discovered for t in rows] == np.cumsum(hist).tolist()
        assert [t.e_frontier for t in rows] == (ehist.tolist() if arcs else [-1] * len(hist))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("kernel", ALL_KERNELS, ids=gsw.KERNEL_NAMES)
def test_fixed_kernel_parity(name, kernel):
    g, G, srcs, refs, comp = case(name)
    arcs = kernel % 2 == 0  # half the runs also count the frontier arcs
    lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=kernel, count_arcs=arcs)
    assert all(t.kernel == kernel for t in trace)
    _check_result(g, srcs, refs, comp, lv, pa, trace, arcs)


@pytest.mark.parametrize("name", list(CASES))
def test_random_schedules(name):
    g, G, srcs, refs, comp = case(name)
    rng = np.random.default_rng(1234)
    depth = max(len(r[2]) for r in refs)
    for trial in range(6):
        sched = rng.integers(0, gsw.N_KERNELS, size=depth).astype(np.int32)
        arcs = trial % 2 == 1
        lv, pa, trace = gsw.bfs(G, srcs, policy="schedule", schedule=sched, count_arcs=arcs)
        for t in trace:
            assert t.kernel == sched[min(t.level, depth - 1)]
        _check_result(g, srcs, refs, comp, lv, pa, trace, arcs)


def _handmade_tree():
    # split on the frontier fraction, then on the discovered fraction
    return dict(
        left=[1, 3, 5, -1, -1, -1, -1], right=[2, 4, 6, -1, -1, -1, -1],
        feature=[21, 23, 23, -2, -2, -2, -2], threshold=[0.01, 0.5, 0.9, -2, -2, -2, -2],
        value=[[1, 1, 1, 1], [3, 1, 0, 0], [0, 0, 2, 1], [0, 4, 0, 0], [5, 0, 0, 0],
               [0, 0, 6, 0], [0, 0, 1, 1]],
        class_kernel=[gsw.PUSH_WAVE32, gsw.PUSH_VERTEX, gsw.PULL_BITMAP, gsw.PUSH_EDGE])


@pytest.mark.parametrize("name", ["rmat10", "rmat14", "er_ragged", "grid", "chunglu", "star"])
def test_tree_policy_matches_oracle_walk(name):
    g, G, srcs, refs, comp = case(name)
    T = _handmade_tree()
    tree = gsw.Tree(T)
    lv, pa, trace = gsw.bfs(G, srcs, policy="tree", tree=tree)
    _check_result(g, srcs, refs, comp, lv, pa, trace)
    gf = ofeat.graph_features(g.offs)
    for i in range(len(srcs)):
        hist = refs[i][2]
        prev = gsw.DEFAULT_KERNEL
        for t in [t for t in trace if t.source_idx == i]:
            x = ofeat.level_features(g.offs, hist, t.level, gf)
            k, unknown = otree.predict(T, x, prev, t.level, gsw.DEFAULT_KERNEL)
            assert t.kernel == k and bool(t.flags & 1) == unknown
            prev = k


def _big_tree(depth=9, seed=17):
    # complete binary tree (children 2i+1, 2i+2) on random features and
    # thresholds near the features' ranges; leaves with a random class, a few tied
    rng = np.random.default_rng(seed)
    n_int = 2 ** depth - 1
    n = 2 ** (depth + 1) - 1
    left = [2 * i + 1 if i < n_int else -1 for i in range(n)]
    right = [2 * i + 2 if i < n_int else -1 for i in range(n)]
    feature = [int(rng.choice([20, 21, 22, 23])) if i < n_int else -2 for i in range(n)]
    thr = []
    for i in range(n):
        f = feature[i]
        thr.append(-2.0 if i >= n_int else float(rng.uniform(0, 1) if f in (21, 23) else rng.uniform(0, 3000)))
    kernels = [gsw.PUSH_VERTEX, gsw.PUSH_WAVE8, gsw.PUSH_EDGE, gsw.PULL_BITMAP,
               gsw.kernel_id(gsw.REV_EDGE_SCAN), gsw.kernel_id(gsw.PUSH_VERTEX, gsw.COUNT_THREAD)]
    value = []
    for i in range(n):
        v = [0.0] * len(kernels)
        if i >= n_int:
            v[int(rng.integers(len(kernels)))] = 3.0
            if rng.random() < 0.1:
                v[(int(np.argmax(v)) + 1) % len(kernels)] = 3.0
        else:
            v = [1.0] * len(kernels)
        value.append(v)
    return dict(left=left, right=right, feature=feature, threshold=thr, value=value, class_kernel=kernels)


@pytest.mark.parametrize("which", ["shipped", "mid", "big", "huge"])
@pytest.mark.parametrize("name", ["rmat14", "grid", "chunglu"])
def test_device_tree_walk_matches_oracle(name, which):
    # the device copy of the tree is specialised to the graph and evaluated
    # by one wave (up to 256 nodes, four per lane: the 255-node tree), by the
    # last workgroup into an LDS table (up to 2048: the 1023-node tree) or
    # walked in global memory (the 4095-node tree); every level's choice
    # equals the oracle's walk of the whole tree
    import json

    g, G, srcs, refs, comp = case(name)
    if which == "shipped":
        from paper_1708_01159_amd import trees

        T = json.load(open(trees.default_path()))
        tree = trees.load_default()
    else:
        T = _big_tree(depth={"mid": 7, "big": 9, "huge": 11}[which])
        tree = gsw.Tree(T)
    assert len(T["left"]) > {"shipped": 50, "mid": 192, "big": 512, "huge": 2048}[which]
    lv, pa, trace = gsw.bfs(G, srcs, policy="tree", tree=tree)
    _check_result(g, srcs, refs, comp, lv, pa, trace)
    gf = ofeat.graph_features(g.offs)
    for i in range(len(srcs)):
        hist = refs[i][2]
        prev = gsw.DEFAULT_KERNEL
        for t in [t for t in trace if t.source_idx == i]:
            x = ofeat.level_features(g.offs, hist, t.level, gf)
            k, unknown = otree.predict(T, x, prev, t.level, gsw.DEFAULT_KERNEL)
            assert t.kernel == k and bool(t.flags & 1) == unknown, (t.level, t.kernel, k)
            prev = k


def test_level_features_match_oracle():
    g, G, srcs, refs, comp = case("rmat14")
    hist = refs[0][2]
    gf = ofeat.graph_features(g.offs)
    for d in range(len(hist)):
        want = ofeat.level_features(g.offs, hist, d, gf)
        got = G.level_features(int(hist[d]), int(hist[: d + 1].sum()))
        np.testing.assert_allclose(got, want, rtol=1e-12)
        exact = [0, 1, 2, 3, 4, 5, 6, 20, 22]
        assert np.array_equal(got[exact], want[exact])


def _canonical(g, lv):
    par = np.full(g.n, -1, dtype=np.int64)
    rows = np.repeat(np.arange(g.n), g.degrees())
    ok = (lv[rows] > 0) & (lv[g.cols] == lv[rows] - 1)
    cand = np.full(g.n, np.iinfo(np.int64).max)
    np.minimum.at(cand, rows[ok], g.cols[ok].astype(np.int64))
    has = lv > 0
    par[has] = cand[has]
    par[lv == 0] = np.flatnonzero(lv == 0)
    return par


@pytest.mark.parametrize("name", ["rmat14", "grid", "dirty", "disjoint"])
def test_canonical_parents_exact(name):
    g, G, srcs, refs, comp = case(name)
    for kernel in (gsw.PUSH_VERTEX, gsw.PULL_BITMAP, gsw.PUSH_EDGE):
        lv, pa, _ = gsw.bfs(G, srcs, policy="fixed", kernel=kernel, canonical_parents=True)
        for i in range(len(srcs)):
            assert np.array_equal(pa[i], _canonical(g, refs[i][0]))


def _probe_positions_graph():
    # source 0 -> frontier F = 1000..1099 (depth 1) -> targets 2000 + k
    # (depth 2).  Target k's sorted row holds k fillers (ids 1..k, reached only
    # through targets), then two members of F, then five trailing fillers
    # (ids 3000..3004): its first frontier neighbour sits at row position k,
    # across the head copy (4 arcs), the eager probes (next 8) and the wave
    # scan's 64-arc chunks that follow.
    src, dst = [], []
    for f in range(1000, 1100):
        src.append(0), dst.append(f)
    for k in range(150):
        t = 2000 + k
        for j in range(1, k + 1):
            src.append(t), dst.append(j)
        for f in (1000 + k % 100, 1000 + (k + 7) % 100):
            src.append(t), dst.append(f)
        for j in range(3000, 3005):
            src.append(t), dst.append(j)
    return gg.from_edges(3005, src, dst, symmetrize=True, name="probe_positions")


@pytest.mark.parametrize("name", ["probe_positions", "rmat14", "chunglu", "er_ragged", "grid", "disjoint"])
def test_pull_parent_is_a_frontier_neighbour(name):
    # a bottom-up level probes a vertex's head (its neighbours of largest
    # degree on a skewed degree law -- rmat14, chunglu, disjoint and this
    # graph -- else its first arcs: er_ragged, grid) and then its row,
    # stopping at the first neighbour in the frontier (Section III-A): with
    # pull at every level the
    # levels are exact and every parent is a neighbour one level up, found
    # wherever it sits in the row (the head, the lane's own probes or the
    # wave's scan); canonical parents are the smallest such neighbour
    if name == "probe_positions":
        g = _probe_positions_graph()
        G = gsw.Graph.from_csr(g.offs, g.cols)
        srcs = np.array([0, 2077], dtype=np.int32)
        refs = [oracle.bfs(g.offs, g.cols, int(s)) for s in srcs]
    else:
        g, G, srcs, refs, comp = case(name)
    lv, pa, _ = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PULL_BITMAP)
    for i in range(len(srcs)):
        assert np.array_equal(lv[i], refs[i][0])
        checks.check_bfs(g.offs, g.cols, int(srcs[i]), lv[i], pa[i])
    lv, pa, _ = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PULL_BITMAP, canonical_parents=True)
    for i in range(len(srcs)):
        assert np.array_equal(pa[i], _canonical(g, refs[i][0])), (name, int(srcs[i]))


def _pull_parents_expected(g, lv, ranked):
    """The parent a bottom-up level gives each vertex of depth >= 1: the
    first of its head neighbours one level up, in head order, else the first
    such neighbour in row order.  A ranked head is the four neighbours of
    largest degree among the row's first 256 arcs (an earlier arc first
    among equals), else the head is the row's first four arcs."""
    deg = np.diff(g.offs)
    want = np.full(g.n, -1, dtype=np.int64)
    for v in np.flatnonzero(lv >= 1):
        row = g.cols[g.offs[v]:g.offs[v + 1]]
        up = lv[row] == lv[v] - 1
        if ranked:
            scan = row[:256]
            head = sorted(range(scan.shape[0]), key=lambda e: (-int(deg[scan[e]]), e))[:4]
            hits = [int(scan[e]) for e in head if up[e]]
            if hits:
                want[v] = hits[0]
                continue
        want[v] = int(row[np.argmax(up)])
    return want


@pytest.mark.parametrize("name", ["rmat14", "chunglu", "star", "er_ragged", "grid"])
def test_pull_parents_follow_the_head_rule(name):
    # the library ranks the head exactly where the byte model does (out-degree
    # standard deviation above the mean): with pull at every level every
    # parent is the one the head the rule picks gives
    from paper_1708_01159_amd import traffic

    g, G, srcs, refs, comp = case(name)
    ranked = traffic.head_is_ranked(g.offs)
    assert ranked == (name in ("rmat14", "chunglu", "star"))
    lv, pa, _ = gsw.bfs(G, srcs[:2], policy="fixed", kernel=gsw.PULL_BITMAP)
    for i in range(min(2, len(srcs))):
        assert np.array_equal(lv[i], refs[i][0])
        want = _pull_parents_expected(g, lv[i], ranked)
        m = lv[i] >= 1
        assert np.array_equal(pa[i][m], want[m]), (name, int(srcs[i]))


def test_device_pointers_and_torch_stream():
    import torch

    g, G, srcs, refs, comp = case("rmat14")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PULL_BITMAP, device=True)
    stream.synchronize()
    assert lv.is_cuda and lv.shape == (len(srcs), g.n)
    _check_result(g, srcs, refs, comp, lv.cpu().numpy(), pa.cpu().numpy(), trace)
    # borrowed device CSR
    offs_t = torch.from_numpy(g.offs).cuda()
    cols_t = torch.from_numpy(g.cols).cuda()
    G2 = gsw.Graph.from_csr(offs_t, cols_t)
    lv2, pa2, trace2 = gsw.bfs(G2, srcs, policy="fixed", kernel=gsw.PUSH_EDGE)
    _check_result(g, srcs, refs, comp, lv2, pa2, trace2)
    G2.close()


def test_arc_counts_off_by_default():
    g, G, srcs, refs, comp = case("rmat14")
    lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PULL_BITMAP)
    _check_result(g, srcs, refs, comp, lv, pa, trace, arcs=False)
    from paper_1708_01159_amd import trees

    lv, pa, trace = gsw.bfs(G, srcs, policy="tree", tree=trees.load_default(), count_arcs=True)
    _check_result(g, srcs, refs, comp, lv, pa, trace, arcs=True)


def test_time_levels_and_no_parents():
    g, G, srcs, refs, comp = case("rmat14")
    lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PUSH_WAVE16, parents=False,
                            time_levels=True)
    assert pa is None
    assert all(t.ms >= 0 for t in trace)
    for i in range(len(srcs)):
        assert np.array_equal(lv[i], refs[i][0])


def _directed_cases():
    a = gg.rmat(10, 8, seed=40)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = rows < a.cols  # orient every edge from low id to high id: a DAG
    dag = gg.from_edges(a.n, rows[keep], a.cols[keep], symmetrize=False, name="dag")
    # a random 60% of an R-MAT graph's arcs: cycles, reciprocated and one-way arcs
    b = gg.rmat(12, 8, seed=41)
    brow = np.repeat(np.arange(b.n), b.degrees())
    keep = np.random.default_rng(41).random(b.nnz) < 0.6
    r = gg.from_edges(b.n, brow[keep], b.cols[keep], symmetrize=False, name="rmat12_directed")
    # directed cycle plus chords, ragged n
    n = 1003
    src = list(range(n)) + list(range(0, n, 7))
    dst = [(i + 1) % n for i in range(n)] + [(i * 31 + 5) % n for i in range(0, n, 7)]
    cyc = gg.from_edges(n, src, dst, symmetrize=False, name="cycle")
    return [dag, r, cyc]


@pytest.mark.parametrize("which", [0, 1, 2])
def test_directed_graph_every_kernel(which):
    """Directed graphs: the top-down kernels follow out-arcs, the bottom-up and
    reverse-edge-list kernels the transpose the library keeps; every kernel
    (and count variant) equals the oracle, parents pass the directed
    invariants, and the trace's e_f equals the out-degree sums."""
    d = _directed_cases()[which]
    G = gsw.Graph.from_csr(d.offs, d.cols)
    assert not G.symmetric
    srcs = np.flatnonzero(d.degrees() > 0)[:2].astype(np.int32)
    refs = [oracle.bfs(d.offs, d.cols, int(s)) for s in srcs]
    for k in ALL_KERNELS:
        lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=k, count_arcs=True)
        for i, s in enumerate(srcs):
            assert np.array_equal(lv[i], refs[i][0]), (gsw.KERNEL_NAMES[k], int(s))
            checks.check_bfs_directed(d.offs, d.cols, int(s), lv[i], pa[i])
            rows = [t for t in trace if t.source_idx == i]
            assert [t.e_frontier for t in rows] == refs[i][3].tolist()
        # canonical parents on a directed graph: the smallest in-neighbour one level up
        lv, pa, _ = gsw.bfs(G, srcs, policy="fixed", kernel=k, canonical_parents=True)
        for i in range(len(srcs)):
            assert np.array_equal(pa[i], _canonical_directed(d, refs[i][0]))
    tr = gsw.Tree.constant(gsw.PULL_BITMAP)
    lv, _, trace = gsw.bfs(G, srcs, policy="tree", tree=tr)
    for i in range(len(srcs)):
        assert np.array_equal(lv[i], refs[i][0])
    assert all(t.kernel == gsw.PULL_BITMAP and not t.flags & 2 for t in trace)
    G.close()


def _canonical_directed(g, lv):
    rows = np.repeat(np.arange(g.n), g.degrees())
    par = np.full(g.n, -1, dtype=np.int64)
    ok = (lv[rows] >= 0) & (lv[g.cols] == lv[rows] + 1)  # arc u -> v one level down
    cand = np.full(g.n, np.iinfo(np.int64).max)
    np.minimum.at(cand, g.cols[ok].astype(np.int64), rows[ok])
    has = lv > 0
    par[has] = cand[has]
    par[lv == 0] = np.flatnonzero(lv == 0)
    return par


def test_error_paths():
    g, G, srcs, refs, comp = case("rmat10")
    with pytest.raises(gsw.GswError) as ei:
        gsw.bfs(G, [g.n], policy="fixed", kernel=0)
    assert ei.value.status == gsw.EINVAL
    with pytest.raises(gsw.GswError) as ei:
        gsw.bfs(G, [0], policy="fixed", kernel=gsw.N_KERNELS)
    assert ei.value.status == gsw.EINVAL
    o = gsw.BfsOpts()
    gsw.lib().gsw_bfs_opts_default(o)
    lv = np.empty(g.n, dtype=np.int32)
    src = np.array([0], dtype=np.int32)
    st = gsw.lib().gsw_bfs(G.handle, src.ctypes.data, 1, lv.ctypes.data, None, None, 0, None, o)
    assert st == gsw.ENOTREE
    # a result is still right after the errors
    lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PUSH_EDGE)
    _check_result(g, srcs, refs, comp, lv, pa, trace)


def test_profile_api():
    g, G, srcs, refs, comp = case("rmat14")
    s = int(srcs[0])
    times, frontier, ks = gsw.bfs_profile(G, s, reps=3)
    hist = refs[0][2]
    assert times.shape == (len(hist), gsw.N_KERNELS)  # every base kernel in every count variant
    assert np.array_equal(frontier, hist)
    assert np.all(times > 0)
    # the profiled state is left consistent: a normal BFS afterwards is exact
    lv, pa, trace = gsw.bfs(G, srcs, policy="fixed", kernel=gsw.PUSH_VERTEX)
    _check_result(g, srcs, refs, comp, lv, pa, trace)


def test_graph_info():
    g, G, srcs, refs, comp = case("rmat14")
    info = G.info()
    assert info["n"] == g.n and info["nnz"] == g.nnz
    np.testing.assert_allclose(info["deg_stats"], ofeat.graph_features(g.offs)[2:8], rtol=1e-12)
    assert info["dev_bytes"] >= 8 * (g.n + 1) + 4 * g.nnz


@pytest.mark.parametrize("width", [3000, 300])
def test_push_edge_empty_and_long_rows(width):
    # directed: the source reaches `width` vertices, most without out-arcs
    # and every (width/10)-th with a row of 2000, so push_edge's chunks span
    # runs of empty queue entries and rows longer than a chunk; then the same
    # graph made symmetric (a 3000-entry frontier of mostly one-arc rows spans
    # more entries per chunk than the staging window holds).  300 entries
    # take the one-launch form, 3000 the two-launch one.
    hubs = list(range(1, width + 1, width // 10))
    src = [0] * width + [h for h in hubs for _ in range(2000)]
    dst = list(range(1, width + 1)) + [width + 1 + i * 2000 + j for i in range(len(hubs)) for j in range(2000)]
    n = width + 1 + 2000 * len(hubs)
    for sym in (False, True):
        d = gg.from_edges(n, src, dst, symmetrize=sym)
        G = gsw.Graph.from_csr(d.offs, d.cols, flags=gsw.ASSUME_SYMMETRIC if sym else 0)
        for s in (0, 1):
            ref = oracle.levels(d.offs, d.cols, s)
            lv, pa, _ = gsw.bfs(G, [s], policy="fixed", kernel=gsw.PUSH_EDGE)
            assert np.array_equal(lv[0], ref), (sym, s)
            if sym:
                checks.check_bfs(d.offs, d.cols, s, lv[0], pa[0], checks.components(d.n, d.offs, d.cols))
        G.close()


@pytest.mark.parametrize("cap", [1, 3])
@pytest.mark.parametrize("name", ["rmat14", "star", "er_ragged"])
def test_launches_smaller_than_levels(name, cap):
    # every level launch capped at 1 or 3 workgroups: each kernel's levels
    # then ask for more workgroups than they get and stride over their work
    # (pull over all words, push_edge's prefix blocks and arc slices, the
    # queue-driven kernels' rounds); results are unchanged
    g, G, srcs, refs, comp = case(name)
    for k in ALL_KERNELS:
        lv, pa, trace = gsw.bfs(G, srcs[:2], policy="fixed", kernel=k, max_workgroups=cap)
        _check_result(g, srcs[:2], refs[:2], comp, lv, pa, trace)
    from paper_1708_01159_amd import trees

    lv, pa, trace = gsw.bfs(G, srcs[:2], policy="tree", tree=trees.load_default(), max_workgroups=cap)
    _check_result(g, srcs[:2], refs[:2], comp, lv, pa, trace)
