"""Create/destroy cycles: 10^4 graphs (some with their single-source and
components workspaces allocated, some with a session), and 10^4 trees, leave
device memory and host memory where they started."""
import numpy as np
import pytest

from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw, trees

pytestmark = pytest.mark.gpu


def _cycle(g, tree, i):
    G = gsw.Graph.from_csr(g.offs, g.cols)
    if i % 50 == 0:
        gsw.bfs(G, [1], policy="tree", tree=tree)
        gsw.components(G, tree=tree)
        s = gsw.Session(G, 64)
        s.close()
    G.close()


def test_ten_thousand_create_destroy_cycles_do_not_leak():
    import psutil
    import torch

    g = gg.rmat(8, 8, seed=3)
    tree = trees.load_default()
    proc = psutil.Process()
    for i in range(200):  # first-use allocations (runtime, caches) before the baseline
        _cycle(g, tree, i)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    rss0 = proc.memory_info().rss
    for i in range(10000):
        _cycle(g, tree, i)
    for _ in range(10000):
        t = gsw.Tree.load(trees.default_path())
        del t  # destroyed by its finaliser
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    rss1 = proc.memory_info().rss
    assert free0 - free1 < (32 << 20), "device memory fell by %d bytes" % (free0 - free1)
    assert rss1 - rss0 < (64 << 20), "host memory grew by %d bytes" % (rss1 - rss0)
