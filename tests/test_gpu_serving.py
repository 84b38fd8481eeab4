"""GPU: continuously batched serving sessions.  Every query's levels equal
the CPU oracle's and the same query run alone through gsw_bfs, whether it
ran alone or among many others admitted at different times."""
import numpy as np
import pytest

import oracle
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import gsw, serve

pytestmark = pytest.mark.gpu

_cache = {}


def resident(name):
    if name not in _cache:
        g = {"rmat12": lambda: gg.rmat(12, 16, seed=71),
             "grid": lambda: gg.grid(60, 45, 0.05, seed=72),
             "er": lambda: gg.erdos_renyi(30011, 60000, seed=73)}[name]()
        G = gsw.Graph.from_csr(g.offs, g.cols)
        _cache[name] = (g, G)
    return _cache[name]


def alone(G, s):
    return gsw.bfs(G, [int(s)], policy="fixed", kernel=gsw.PUSH_EDGE, parents=False)[0][0]


def test_session_results_and_slot_reuse():
    g, G = resident("rmat12")
    sess = gsw.Session(G, slots=4)
    srcs = gg.pick_sources(g, 10, 3)
    got = {}
    it = iter(srcs)
    slot_src = {}
    for _ in range(200):
        for s in it:
            k = sess.admit(int(s))
            if k is None:
                it = iter([s] + list(it))
                break
            slot_src[k] = int(s)
        fin, _ = sess.step(2)
        for k in fin:
            got[slot_src.pop(k)] = sess.fetch(k)
        if len(got) == len(srcs):
            break
    assert len(got) == len(srcs)
    for s, lv in got.items():
        assert np.array_equal(lv, oracle.levels(g.offs, g.cols, s))
    sess.close()


def test_session_busy_and_mid_flight_admission():
    g, G = resident("grid")
    sess = gsw.Session(G, slots=2)
    a, b, c = gg.pick_sources(g, 3, 9).tolist()
    ka = sess.admit(a)
    sess.step(3)  # a is mid-traversal (the grid is deep)
    kb = sess.admit(b)
    assert sess.admit(c) is None  # both slots busy
    res = {}
    while len(res) < 2:
        fin, _ = sess.step(5)
        for k in fin:
            res[k] = sess.fetch(k)
    assert np.array_equal(res[ka], oracle.levels(g.offs, g.cols, a))
    assert np.array_equal(res[kb], oracle.levels(g.offs, g.cols, b))
    kc = sess.admit(c)
    assert kc is not None
    while True:
        fin, _ = sess.step(50)
        if fin:
            break
    assert np.array_equal(sess.fetch(kc), oracle.levels(g.offs, g.cols, c))


def test_session_isolated_source_and_thresholds():
    a = gg.rmat(9, 8, seed=74)
    g = gg.from_edges(a.n + 2, np.repeat(np.arange(a.n), a.degrees()), a.cols)
    G = gsw.Graph.from_csr(g.offs, g.cols)
    for p2p in ((0.0, 0.0), (1e9, 1e9)):
        sess = gsw.Session(G, slots=70)
        sess.set_thresholds(*p2p)
        srcs = [g.n - 1] + gg.pick_sources(g, 65, 11).tolist()
        slots = [sess.admit(s) for s in srcs]
        res = {}
        while len(res) < len(srcs):
            fin, _ = sess.step(4)
            for k in fin:
                res[k] = sess.fetch(k)
        for s, k in zip(srcs, slots):
            assert np.array_equal(res[k], oracle.levels(g.offs, g.cols, s)), s


def test_session_join_while_others_pull():
    # queries admitted while the first ones are in their bottom-up levels run
    # top-down themselves in the same passes, and still match the oracle
    g, G = resident("rmat12")
    sess = gsw.Session(G, slots=40)
    first = gg.pick_sources(g, 16, 12).tolist()
    later = gg.pick_sources(g, 16, 13).tolist()
    slot_src = {sess.admit(s): s for s in first}
    res = {}
    fin, _ = sess.step(2)
    for k in fin:
        res[slot_src[k]] = sess.fetch(k)
    for s in later:
        slot_src[sess.admit(s)] = s
    while len(res) < len(set(first + later)):
        fin, run = sess.step(100)
        assert run > 0 or fin
        for k in fin:
            res[slot_src.pop(k)] = sess.fetch(k)
    for s, lv in res.items():
        assert np.array_equal(lv, oracle.levels(g.offs, g.cols, s)), s
    sess.close()


def test_session_heavy_rows_all_push_and_default():
    from test_gpu_msbfs import hub_graph

    g = hub_graph()
    G = gsw.Graph.from_csr(g.offs, g.cols)
    hubs = list(range(g.n - 3, g.n))
    srcs = hubs + gg.pick_sources(g, 30, 62).tolist()
    for p2p in ((1e9, 1e9), None):
        sess = gsw.Session(G, slots=16)
        if p2p:
            sess.set_thresholds(*p2p)
        todo = list(srcs)
        slot_src, res = {}, {}
        while len(res) < len(set(srcs)):
            while todo:
                k = sess.admit(todo[0])
                if k is None:
                    break
                slot_src[k] = todo.pop(0)
            fin, _ = sess.step(3)
            for k in fin:
                res[slot_src.pop(k)] = sess.fetch(k)
        for s in srcs:
            assert np.array_equal(res[s], oracle.levels(g.offs, g.cols, s)), s
        sess.close()
    G.close()


@pytest.mark.parametrize("solo", [False, True])
def test_server_mix_equals_alone(solo):
    names = ["rmat12", "grid", "er"]
    residents = {}
    cands = {}
    for nm in names:
        g, G = resident(nm)
        residents[nm] = serve.Resident(nm, G, serve.component_edges(g.offs, g.cols))
        cands[nm] = np.flatnonzero(g.degrees() > 0)
    # 96 queries arriving within 30 ms: they overlap on the device
    trace = serve.poisson_trace(3200.0, 0.03, names, cands, seed=5)
    assert len(trace) >= 64 and len({t[1] for t in trace}) == 3
    srv = serve.Server(residents, slots=64, levels_per_step=3, keep_levels=True, solo=solo)
    qs = srv.run(trace)
    assert (srv.solo_served > 0) == solo
    assert all(q.t_done >= q.t_arrival for q in qs)
    for q in qs:
        g, G = resident(q.graph)
        ref = oracle.levels(g.offs, g.cols, q.source)
        assert np.array_equal(q.levels, ref), (q.graph, q.source)
        assert np.array_equal(q.levels, alone(G, q.source)), (q.graph, q.source)
    stats = serve.summarize(qs, residents, "batched")
    assert stats["queries"] == len(trace) and stats["p99_ms"] >= stats["p50_ms"] > 0


def test_server_tiny_budget_queues_instead_of_failing():
    names = ["rmat12", "grid"]
    residents = {nm: serve.Resident(nm, resident(nm)[1],
                                    serve.component_edges(resident(nm)[0].offs, resident(nm)[0].cols))
                 for nm in names}
    cands = {nm: np.flatnonzero(resident(nm)[0].degrees() > 0) for nm in names}
    trace = serve.poisson_trace(2000.0, 0.02, names, cands, seed=6)
    # room for one session at a time: the other graph's queries wait for eviction
    budget = max(serve.session_bytes(resident(nm)[1], 8) for nm in names) + 1
    srv = serve.Server(residents, slots=8, hbm_budget=budget, keep_levels=True)
    qs = srv.run(trace)
    for q in qs:
        g, _ = resident(q.graph)
        assert np.array_equal(q.levels, oracle.levels(g.offs, g.cols, q.source))
    assert srv.evictions >= 1


def test_session_bytes_are_what_the_session_holds():
    g, G = resident("er")
    for slots in (1, 64, 65, 300):
        sess = gsw.Session(G, slots=slots)
        assert sess.info()["dev_bytes"] == G.session_bytes(slots)
        sess.close()
    before = G.info()["dev_bytes"]
    if before < G.workspace_bytes():  # workspace not built yet on this graph
        gsw.bfs(G, [0], policy="fixed", kernel=gsw.PUSH_EDGE)
        assert G.info()["dev_bytes"] - before == G.workspace_bytes()


def test_session_counter_past_2_31():
    """The session's level counter is 64-bit: queries that start just below
    2^31 and run across it keep exact levels (start and level arithmetic,
    the record ring's slot and tag)."""
    g, G = resident("grid")  # deep: ~100 levels per query
    sess = gsw.Session(G, slots=8)
    sess.rebase((1 << 31) - 40)
    assert sess.info()["iteration"] == (1 << 31) - 40
    srcs = gg.pick_sources(g, 12, 21).tolist()
    todo, slot_src, res = list(srcs), {}, {}
    while len(res) < len(set(srcs)):
        while todo:
            k = sess.admit(todo[0])
            if k is None:
                break
            slot_src[k] = todo.pop(0)
        fin, _ = sess.step(7)
        for k in fin:
            res[slot_src.pop(k)] = sess.fetch(k)
    assert sess.info()["iteration"] > (1 << 31) + 20
    for s, lv in res.items():
        assert np.array_equal(lv, oracle.levels(g.offs, g.cols, s)), s
    # rebase refuses while a query runs
    k = sess.admit(srcs[0])
    sess.step(1)
    with pytest.raises(gsw.GswError) as ei:
        sess.rebase(0)
    assert ei.value.status == gsw.EBUSY
    while True:
        fin, _ = sess.step(50)
        if fin:
            break
    sess.fetch(k)
    sess.rebase(5)
    k = sess.admit(srcs[1])
    while True:
        fin, _ = sess.step(50)
        if fin:
            break
    assert np.array_equal(sess.fetch(k), oracle.levels(g.offs, g.cols, srcs[1]))
    sess.close()


def test_session_cancel_running_and_admitted():
    """A running query cancelled mid-traversal stops at the next boundary and
    its slot is freed without being reported; one cancelled before it starts
    is dropped at once; both slots then serve new queries exactly (the
    cancelled query's partial row was cleared)."""
    g, G = resident("grid")  # ~100 levels per query
    sess = gsw.Session(G, slots=2)
    a, b, c = gg.pick_sources(g, 3, 31).tolist()
    ka = sess.admit(a)
    fin, run = sess.step(3)
    assert not fin and run == 3  # a is mid-traversal
    assert sess.cancel(ka)
    kb = sess.admit(b)
    assert kb is not None and kb != ka
    assert sess.cancel(kb) and not sess.cancel(kb)
    while True:
        fin, run = sess.step(50)
        assert not fin  # a cancelled query is never reported finished
        if run == 0:
            break
    assert sess.info()["busy"] == 0
    ks = {sess.admit(c): c, sess.admit(a): a}
    assert set(ks) == {0, 1}
    res = {}
    while len(res) < 2:
        fin, _ = sess.step(50)
        for k in fin:
            res[k] = sess.fetch(k)
    for k, s in ks.items():
        assert np.array_equal(res[k], oracle.levels(g.offs, g.cols, s)), s
    assert not sess.cancel(0)  # nothing admitted any more
    sess.close()


def test_session_created_while_the_default_stream_is_busy():
    """A session's device state is initialised on the session's own stream:
    one created while the process's default stream still has work queued
    (a bounded spin kernel) answers its queries exactly.  Initialising it on
    the default stream, which the session's non-blocking stream does not wait
    for, would let that work land after the session's first levels and reset
    its level counter."""
    import torch

    g, G = resident("rmat12")
    srcs = gg.pick_sources(g, 6, 11)
    for rep in range(3):
        torch.cuda._sleep(20_000_000)  # a few ms of spinning on the default stream
        sess = gsw.Session(G, slots=8)
        got, slot_src = {}, {}
        for s in srcs:
            slot_src[sess.admit(int(s))] = int(s)
        for _ in range(100):
            fin, run = sess.step(64)
            for k in fin:
                got[slot_src.pop(k)] = sess.fetch(k)
            if not slot_src:
                break
        assert sorted(got) == sorted(int(s) for s in srcs)
        for s, lv in got.items():
            assert np.array_equal(lv, oracle.levels(g.offs, g.cols, s)), (rep, s)
        sess.close()
        torch.cuda.synchronize()
