"""Full-size parity in the launch configurations the benchmark times:
R-MAT scale 22 with the shipped tree (sampled sources: levels bit-exact
against the oracle, parents through the invariants), the batched search at
scale 20 with 1024 sources (sampled rows), and one source of each
structure-sweep graph."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw, trees

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat22():
    g = gg.workload("rmat22")
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    yield g, G
    G.close()


def test_rmat22_tree_switched_sampled_sources(rmat22):
    import torch

    g, G = rmat22
    k, seed = gg.WORKLOAD_SOURCES["rmat22"]
    srcs = gg.pick_sources(g, k, seed)
    lv = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
    pa = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
    r = gsw.Runner(G, lv, pa, policy="tree", tree=trees.load_default(), time_levels=True)
    comp = None
    for i in (0, 37):
        s = int(srcs[i])
        r.run(s)
        got = lv[0].cpu().numpy()
        ref, _, hist, _ = oracle.bfs(g.offs, g.cols, s)
        assert np.array_equal(got, ref), "source %d" % s
        rows = r.rows()
        assert [t.n_frontier for t in rows] == hist.tolist()
        assert len({t.kernel for t in rows}) >= 2  # the tree switched kernels
        if i == 0:
            comp = checks.components(g.n, g.offs, g.cols)
            checks.check_bfs(g.offs, g.cols, s, got, pa[0].cpu().numpy(), comp)


def test_rmat22_every_fixed_kernel_one_source(rmat22):
    g, G = rmat22
    s = int(gg.pick_sources(g, 64, 102)[5])
    ref = oracle.levels(g.offs, g.cols, s)
    for k in (gsw.PUSH_EDGE, gsw.PULL_BITMAP, gsw.EDGE_SCAN, gsw.PUSH_WAVE64):
        lv, _, _ = gsw.bfs(G, [s], policy="fixed", kernel=k, parents=False)
        assert np.array_equal(lv[0], ref), gsw.KERNEL_NAMES[k]


def test_rmat20_batched_1024_sampled_rows():
    import torch

    g = gg.workload("rmat20")
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    srcs = gg.pick_sources(g, 1024, 106)
    out = torch.empty((1024, g.n), dtype=torch.int8, device="cuda")
    gsw.msbfs(G, srcs, out=out)
    torch.cuda.synchronize()
    for i in (0, 63, 64, 511, 1023):
        ref = oracle.levels(g.offs, g.cols, int(srcs[i]))
        assert np.array_equal(out[i].cpu().numpy().astype(np.int32), ref), i
    G.close()


@pytest.mark.parametrize("name", ["grid2048_del5", "chunglu23", "er22"])
def test_sweep_graph_one_source(name):
    import torch

    g = gg.workload(name)
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    k, seed = gg.WORKLOAD_SOURCES[name]
    s = int(gg.pick_sources(g, k, seed)[0])
    lv = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
    r = gsw.Runner(G, lv, None, policy="tree", tree=trees.load_default(), trace_cap=1 << 16)
    r.run(s)
    assert np.array_equal(lv[0].cpu().numpy(), oracle.levels(g.offs, g.cols, s))
    G.close()
