"""GPU parity of the batched multi-source BFS: every source's int8 levels
equal the CPU oracle's levels bit-exactly; a depth beyond the int8 cap is a
range error, never a truncation."""
import numpy as np
import pytest

import oracle
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw

pytestmark = pytest.mark.gpu

_cache = {}


def graph(name):
    if name not in _cache:
        g = {"rmat12": lambda: gg.rmat(12, 16, seed=51),
             "er_ragged": lambda: gg.erdos_renyi(20011, 50000, seed=52),
             "grid": lambda: gg.grid(40, 37, 0.05, seed=53),
             "chunglu": lambda: gg.chung_lu(8000, 2.1, 10.0, seed=54)}[name]()
        _cache[name] = (g, gsw.Graph.from_csr(g.offs, g.cols))
    return _cache[name]


def expected(g, srcs):
    lv, ok = oracle.msbfs_levels(g.offs, g.cols, srcs)
    assert ok
    return lv


@pytest.mark.parametrize("name", ["rmat12", "er_ragged", "grid", "chunglu"])
@pytest.mark.parametrize("nsrc", [1, 5, 64, 65, 200, 300])
def test_msbfs_matches_oracle(name, nsrc):
    g, G = graph(name)
    srcs = gg.pick_sources(g, nsrc, 1000 + nsrc)
    lv, nl = gsw.msbfs(G, srcs)
    assert lv.shape == (len(srcs), g.n) and lv.dtype == np.int8
    exp = expected(g, srcs)
    for i in range(len(srcs)):
        assert np.array_equal(lv[i], exp[i]), "source index %d (%d)" % (i, srcs[i])


@pytest.mark.parametrize("p2p", [(0.0, 0.0), (1e9, 1e9), (0.01, 0.005)])
def test_msbfs_directions(p2p):
    # all-pull, all-push and a switching run give the same levels
    g, G = graph("rmat12")
    srcs = gg.pick_sources(g, 130, 77)
    lv, _ = gsw.msbfs(G, srcs, push_to_pull=p2p[0], pull_to_push=p2p[1])
    exp = expected(g, srcs)
    assert np.array_equal(lv, exp)


def test_msbfs_sources_in_different_directions():
    # a deep grid and an R-MAT graph side by side: in the same level the
    # R-MAT sources have large frontiers (bottom-up) while the grid sources
    # still push, and the R-MAT hubs take the whole-wave row walk
    a = gg.rmat(11, 16, seed=55)
    b = gg.grid(50, 50, 0.0, seed=56)
    src = np.concatenate([np.repeat(np.arange(a.n), a.degrees()), a.n + np.repeat(np.arange(b.n), b.degrees())])
    dst = np.concatenate([a.cols, a.n + b.cols])
    g = gg.from_edges(a.n + b.n, src, dst)
    G = gsw.Graph.from_csr(g.offs, g.cols)
    assert np.diff(g.offs).max() > 64
    srcs = np.concatenate([gg.pick_sources(a, 70, 57), a.n + gg.pick_sources(b, 70, 58)])
    for p2p in ((0.05, 0.01), (0.002, 0.0005)):
        lv, _ = gsw.msbfs(G, srcs, push_to_pull=p2p[0], pull_to_push=p2p[1])
        assert np.array_equal(lv, expected(g, srcs))


def hub_graph():
    # R-MAT plus three hubs of 2500-3000 arcs: rows past the whole-wave limit
    # go through the chunk list when pushed
    a = gg.rmat(12, 16, seed=59)
    rng = np.random.default_rng(60)
    hs, hd = [], []
    for h, deg in zip(range(3), (2500, 2800, 3000)):
        nb = rng.choice(a.n, size=deg, replace=False)
        hs.append(np.full(deg, a.n + h))
        hd.append(nb)
    src = np.concatenate([np.repeat(np.arange(a.n), a.degrees())] + hs)
    dst = np.concatenate([a.cols] + hd)
    return gg.from_edges(a.n + 3, src, dst)


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("p2p", [(1e9, 1e9), (0.002, 0.0005), (0.0, 0.0)])
def test_msbfs_heavy_rows(p2p, use_graph):
    g = hub_graph()
    G = gsw.Graph.from_csr(g.offs, g.cols)
    assert np.diff(g.offs).max() > 1024
    hubs = np.arange(g.n - 3, g.n)
    srcs = np.concatenate([hubs, gg.pick_sources(g, 100, 61), [int(g.cols[g.offs[g.n - 1]])]])
    lv, _ = gsw.msbfs(G, srcs, push_to_pull=p2p[0], pull_to_push=p2p[1], use_graph=use_graph)
    assert np.array_equal(lv, expected(g, srcs))
    G.close()


def test_msbfs_graph_replays_across_calls():
    # the captured two-level graph is reused by later calls of the same width
    # and recaptured when the width changes; direct launches interleave
    g, G = graph("chunglu")
    for i, (nsrc, use_graph) in enumerate([(64, True), (40, True), (64, False), (130, True), (3, True),
                                           (64, True)]):
        srcs = gg.pick_sources(g, nsrc, 300 + i)
        lv, nl = gsw.msbfs(G, srcs, use_graph=use_graph)
        assert np.array_equal(lv, expected(g, srcs)), (nsrc, use_graph)


def test_msbfs_tiny_graph():
    g = gg.from_edges(5, np.array([0, 1, 2]), np.array([1, 2, 3]))  # path 0-1-2-3, vertex 4 alone
    G = gsw.Graph.from_csr(g.offs, g.cols)
    lv, nl = gsw.msbfs(G, [0, 3, 4, 2])
    assert np.array_equal(lv, expected(g, [0, 3, 4, 2]))
    G.close()


def test_msbfs_1024_sources_device():
    import torch

    g, G = graph("rmat12")
    srcs = gg.pick_sources(g, 1024, 5)
    lv, nl = gsw.msbfs(G, srcs, device=True)
    torch.cuda.synchronize()
    exp = expected(g, srcs)
    assert np.array_equal(lv.cpu().numpy(), exp)


def test_msbfs_repeated_and_isolated_sources():
    a = gg.rmat(9, 8, seed=60)
    g = gg.from_edges(a.n + 3, np.repeat(np.arange(a.n), a.degrees()), a.cols)  # 3 isolated
    G = gsw.Graph.from_csr(g.offs, g.cols)
    s0 = int(np.flatnonzero(g.degrees() > 0)[0])
    srcs = np.array([s0, s0, g.n - 1, s0, g.n - 2], dtype=np.int32)
    lv, _ = gsw.msbfs(G, srcs)
    exp = expected(g, srcs)
    assert np.array_equal(lv, exp)
    assert lv[2, g.n - 1] == 0 and (lv[2] >= 0).sum() == 1


def test_msbfs_directed_graph_push_only():
    a = gg.rmat(10, 8, seed=61)
    rows = np.repeat(np.arange(a.n), a.degrees())
    keep = rows < a.cols
    d = gg.from_edges(a.n, rows[keep], a.cols[keep], symmetrize=False)
    G = gsw.Graph.from_csr(d.offs, d.cols)
    srcs = np.flatnonzero(d.degrees() > 0)[:70].astype(np.int32)
    lv, _ = gsw.msbfs(G, srcs, push_to_pull=0.0)  # pull would be chosen; the graph forbids it
    for i, s in enumerate(srcs):
        ref = oracle.levels(d.offs, d.cols, int(s))
        assert np.array_equal(lv[i].astype(np.int32), ref)


def test_msbfs_level_cap_is_a_range_error():
    n = 200
    p = gg.from_edges(n, list(range(n - 1)), list(range(1, n)))
    G = gsw.Graph.from_csr(p.offs, p.cols)
    with pytest.raises(gsw.GswError) as ei:
        gsw.msbfs(G, [0])
    assert ei.value.status == gsw.ERANGE
    # a source in the middle stays within the cap (eccentricity 100)
    lv, nl = gsw.msbfs(G, [100, 0 + 90])
    assert np.array_equal(lv[0].astype(np.int32), np.abs(np.arange(n) - 100))
    # single-source BFS on the same graph and source still works afterwards
    l2, _, _ = gsw.bfs(G, [0], policy="fixed", kernel=gsw.PUSH_VERTEX)
    assert np.array_equal(l2[0], np.arange(n))


def test_msbfs_bad_arguments():
    g, G = graph("rmat12")
    with pytest.raises(gsw.GswError):
        gsw.msbfs(G, np.arange(1025))
    with pytest.raises(gsw.GswError):
        gsw.msbfs(G, [g.n])


@pytest.mark.parametrize("device", [False, True])
def test_msbfs_fallback_reruns_deep_sources_in_int32(device):
    """A 200-vertex path: sources near an end go deeper than 127.  With the
    fallback they are rerun on the single-source path -- full int32 rows,
    int8 rows holding -128 beyond 127 -- and the other sources keep their
    batched result."""
    import torch

    n = 200
    p = gg.from_edges(n, list(range(n - 1)), list(range(1, n)))
    G = gsw.Graph.from_csr(p.offs, p.cols)
    srcs = np.array([0, 100, 199, 90, 3, 150], dtype=np.int32)
    for tree in (None, gsw.Tree.constant(gsw.PUSH_VERTEX)):
        lv, nl, wide = gsw.msbfs(G, srcs, fallback=True, tree=tree, device=device)
        if device:
            torch.cuda.synchronize()
            lv = lv.cpu().numpy()
            wide = {k: v.cpu().numpy() for k, v in wide.items()}
        # on a path the eccentricity of s is max(s, n - 1 - s): 199, 100, 199, 109, 196, 150
        deep = [i for i, s in enumerate(srcs) if max(int(s), n - 1 - int(s)) > 127]
        assert deep == [0, 2, 4, 5]
        assert sorted(wide) == deep
        for i, s in enumerate(srcs):
            ref = np.abs(np.arange(n) - int(s))
            assert np.array_equal(ref, oracle.levels(p.offs, p.cols, int(s)))
            if i in wide:
                assert np.array_equal(wide[i], ref)
                assert np.array_equal(lv[i].astype(np.int32), np.where(ref > 127, -128, ref))
            else:
                assert np.array_equal(lv[i].astype(np.int32), ref)
    # too little room for the rerun rows is a range error, with the count
    with pytest.raises(gsw.GswError) as ei:
        gsw.msbfs(G, srcs, fallback=True, wide_cap=2)
    assert ei.value.status == gsw.ERANGE
    # nothing past the cap: no rerun (source 72 reaches depth 127 exactly)
    lv, nl, wide = gsw.msbfs(G, [100, 72], fallback=True)
    assert wide == {}
    for i, s in enumerate((100, 72)):
        assert np.array_equal(lv[i].astype(np.int32), np.abs(np.arange(n) - s))
    # one level deeper (source 71 reaches 128) is rerun
    lv, nl, wide = gsw.msbfs(G, [100, 71], fallback=True)
    assert sorted(wide) == [1] and np.array_equal(wide[1], np.abs(np.arange(n) - 71))
    G.close()


@pytest.mark.parametrize("bs", [128, 256, 512])
@pytest.mark.parametrize("use_graph", [True, False])
def test_msbfs_block_sizes(bs, use_graph):
    g = hub_graph()
    G = gsw.Graph.from_csr(g.offs, g.cols)
    srcs = gg.pick_sources(g, 150, 62)
    for p2p in ((0.05, 0.01), (0.0, 0.0), (1e9, 1e9)):
        lv, _ = gsw.msbfs(G, srcs, push_to_pull=p2p[0], pull_to_push=p2p[1], block_size=bs,
                          use_graph=use_graph)
        assert np.array_equal(lv, expected(g, srcs)), (bs, p2p)
    with pytest.raises(gsw.GswError):
        gsw.msbfs(G, srcs, block_size=64)
    G.close()


def test_msbfs_block_size_recapture():
    # the captured graph is remade when the block size changes
    g, G = graph("er_ragged")
    for i, bs in enumerate((256, 512, 512, 128, 256)):
        srcs = gg.pick_sources(g, 70, 400 + i)
        lv, _ = gsw.msbfs(G, srcs, block_size=bs)
        assert np.array_equal(lv, expected(g, srcs)), bs
