"""Serving scheduler on the CPU: a stub session (answers from the oracle, one
simulated level per step) exercises admission, slot reuse, the memory budget
and eviction without a GPU."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1708_01159_amd import graphgen as gg
from paper_1708_01159_amd import serve


class StubGraph:
    def __init__(self, csr):
        self.csr = csr
        self.n = csr.n

    def session_bytes(self, slots):
        return 32 * self.n * ((slots + 63) // 64) + 4 * self.n * slots

    def workspace_bytes(self):
        return 100 * self.n


class StubSession:
    """Same contract as gsw.Session: admit from any thread, step runs until a
    slot finishes or nothing is admitted or running."""

    created = 0

    def __init__(self, graph, slots):
        StubSession.created += 1
        self.g = graph
        self.slots = slots
        self.state = {}  # slot -> [source, start, depth, levels]
        self.pending = {}
        self.it = 0
        self.finished = {}
        self.mu = threading.Lock()

    def admit(self, source):
        with self.mu:
            used = set(self.state) | set(self.pending) | set(self.finished)
            free = [k for k in range(self.slots) if k not in used]
            if not free:
                return None
            self.pending[free[0]] = source
            return free[0]

    def step(self, max_levels):
        fin = []
        for run in range(max_levels):
            with self.mu:  # level boundary: take new admissions
                for k, s in self.pending.items():
                    lv = oracle.levels(self.g.csr.offs, self.g.csr.cols, s)
                    self.state[k] = [s, self.it, int(lv.max()) + 1, lv]
                self.pending = {}
            if not self.state:
                return fin, run
            self.it += 1
            with self.mu:
                for k in list(self.state):
                    s, start, depth, lv = self.state[k]
                    if self.it - start >= depth:
                        fin.append(k)
                        self.finished[k] = lv
                        del self.state[k]
            if fin:
                return fin, run + 1
        return fin, max_levels

    def cancel(self, slot):
        with self.mu:
            if slot in self.pending:
                del self.pending[slot]
                return True
            if slot in self.state:
                del self.state[slot]
                return True
            return False

    def fetch(self, slot, out=None):
        with self.mu:
            lv = self.finished.pop(slot)
        if out is not None:
            out[:] = lv
            return out
        return lv.copy()

    def info(self):
        with self.mu:
            return dict(slots=self.slots, busy=len(self.state) + len(self.pending) + len(self.finished),
                        iteration=self.it, dev_bytes=0)

    def close(self):
        pass


class StubSolo:
    """Single-source lane answered by the oracle."""

    def __init__(self, graph):
        self.g = graph

    def run(self, source, keep):
        lv = oracle.levels(self.g.csr.offs, self.g.csr.cols, source)
        return lv if keep else None


class SlowStubSession(StubSession):
    """A stub whose levels take 0.5 ms each, so deep queries stay running."""

    def step(self, max_levels):
        time.sleep(0.0005)
        return super().step(1)


def make(names):
    res, cands = {}, {}
    graphs = {"a": gg.rmat(9, 8, seed=1), "b": gg.grid(12, 9, 0.0, seed=1), "c": gg.erdos_renyi(700, 900, seed=2),
              "p": gg.from_edges(600, list(range(599)), list(range(1, 600)), name="path600")}
    for nm in names:
        g = graphs[nm]
        res[nm] = serve.Resident(nm, StubGraph(g), serve.component_edges(g.offs, g.cols))
        cands[nm] = np.flatnonzero(g.degrees() > 0)
    return res, cands


def test_scheduler_answers_every_query_correctly():
    res, cands = make(["a", "b", "c"])
    trace = serve.poisson_trace(5000.0, 0.02, ["a", "b", "c"], cands, seed=3)
    srv = serve.Server(res, slots=4, levels_per_step=2, keep_levels=True, session_factory=StubSession)
    qs = srv.run(trace, timeout_s=60)
    assert len(qs) == len(trace)
    for q in qs:
        g = res[q.graph].graph.csr
        assert np.array_equal(q.levels, oracle.levels(g.offs, g.cols, q.source))
        assert q.t_admit >= q.t_arrival and q.t_done >= q.t_admit
    st = serve.summarize(qs, res, "stub")
    assert st["queries"] == len(trace) and st["p99_ms"] >= st["p50_ms"]


def test_solo_lane_takes_queries_of_idle_graphs():
    res, cands = make(["a", "b", "c"])
    # sparse arrivals: most queries find their graph idle; a burst at the end
    # overlaps and goes to the sessions
    trace = serve.poisson_trace(300.0, 0.05, ["a", "b", "c"], cands, seed=8)
    trace += [(0.06, "a", int(cands["a"][i])) for i in range(12)]
    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=StubSession, solo=True,
                       solo_factory=StubSolo)
    qs = srv.run(trace, timeout_s=60)
    assert len(qs) == len(trace)
    for q in qs:
        g = res[q.graph].graph.csr
        assert np.array_equal(q.levels, oracle.levels(g.offs, g.cols, q.source))
    assert 0 < srv.solo_served < len(trace)


def test_budget_forces_eviction_and_queueing():
    res, cands = make(["a", "b"])
    trace = serve.poisson_trace(3000.0, 0.02, ["a", "b"], cands, seed=4)
    budget = max(serve.session_bytes(r.graph, 2) for r in res.values())  # one session fits
    StubSession.created = 0
    srv = serve.Server(res, slots=2, hbm_budget=budget, keep_levels=True, session_factory=StubSession)
    qs = srv.run(trace, timeout_s=60)
    assert all(q.t_done >= 0 for q in qs)
    assert srv.evictions >= 1 and StubSession.created >= 2
    assert srv.used <= budget


def test_poisson_trace_shape():
    res, cands = make(["a", "b", "c"])
    tr = serve.poisson_trace(1000.0, 2.0, ["a", "b", "c"], cands, seed=9)
    ts = np.array([t for t, _, _ in tr])
    assert np.all(np.diff(ts) >= 0) and 1700 < len(tr) < 2300  # ~ rate x duration
    share = np.mean([g == "a" for _, g, _ in tr])
    assert share > np.mean([g == "c" for _, g, _ in tr])  # Zipf: first graph most frequent
    for _, g, s in tr:
        assert s in set(cands[g].tolist())


def test_budget_charges_sessions_lanes_and_workspaces():
    """Server.used is what the sessions and lanes hold: every open session's
    bytes, each open lane's level row, and each lane graph's single-source
    workspace (kept after the lane closes); a lane that does not fit is not
    opened and its queries go to the session."""
    res, cands = make(["a", "b"])
    trace = serve.poisson_trace(300.0, 0.05, ["a", "b"], cands, seed=8)
    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=StubSession, solo=True,
                       solo_factory=StubSolo)
    qs = srv.run(trace, timeout_s=60)
    assert len(qs) == len(trace) and not srv.sessions
    ws = sum(res[nm].graph.workspace_bytes() for nm in srv._ws_charged)
    assert srv._ws_charged and srv.used == ws
    # a budget without room for a lane beside the largest session: every
    # query is served by a session
    ga, gb = res["a"].graph, res["b"].graph
    budget = max(ga.session_bytes(4), gb.session_bytes(4)) + 1
    srv = serve.Server(res, slots=4, hbm_budget=budget, keep_levels=True, session_factory=StubSession,
                       solo=True, solo_factory=StubSolo)
    qs = srv.run(trace, timeout_s=60)
    assert srv.solo_served == 0 and all(q.path == "session" for q in qs)
    assert srv.used <= budget


def test_lanes_never_lock_out_a_session():
    # room for one lane beside the largest session, not two: the second
    # graph's queries still run (in its session)
    res, cands = make(["a", "b"])
    trace = serve.poisson_trace(300.0, 0.05, ["a", "b"], cands, seed=8)
    ga, gb = res["a"].graph, res["b"].graph
    big = max(ga.session_bytes(4), gb.session_bytes(4))
    lane_b = gb.workspace_bytes() + 4 * gb.n
    srv = serve.Server(res, slots=4, hbm_budget=big + lane_b, keep_levels=True, session_factory=StubSession,
                       solo=True, solo_factory=StubSolo)
    qs = srv.run(trace, timeout_s=60)
    assert len(qs) == len(trace) and srv.used <= big + lane_b
    assert {q.graph for q in qs if q.path == "session"} and srv.solo_served > 0


def test_deadline_expires_waiting_and_cancels_running():
    """Deep queries (a 600-vertex path, 0.5 ms per level) on one slot with a
    60 ms deadline: the running one is cancelled, those still waiting expire;
    quick queries on another graph complete with exact levels; percentiles
    count completed queries only."""
    res, cands = make(["a", "p"])
    trace = [(0.001 * i, "p", 0) for i in range(4)] + [(0.002 + 0.001 * i, "a", int(cands["a"][i])) for i in range(6)]
    srv = serve.Server(res, slots=1, levels_per_step=1, keep_levels=True, session_factory=SlowStubSession,
                       deadline_s=0.06)
    qs = srv.run(trace, timeout_s=60)
    by = {}
    for q in qs:
        by.setdefault((q.graph, q.status), []).append(q)
    assert srv.cancelled >= 1
    assert not by.get(("p", "done"))
    assert srv.cancelled + srv.expired == len(qs) - len(by.get(("a", "done"), []))
    for q in by.get(("a", "done"), []):
        g = res["a"].graph.csr
        assert np.array_equal(q.levels, oracle.levels(g.offs, g.cols, q.source))
    for q in qs:
        if q.status != "done":
            assert q.levels is None and q.t_done - q.t_arrival >= 0.06
    st = serve.summarize(qs, res, "deadline")
    assert st["expired"] == srv.expired and st["cancelled"] == srv.cancelled
    assert st["completed"] == len(qs) - srv.expired - srv.cancelled


def test_deadline_expires_queries_that_never_get_a_slot():
    # a budget below any session's size: nothing is ever admitted, every
    # query expires at its deadline instead of the run hanging
    res, cands = make(["a", "b"])
    trace = serve.poisson_trace(1000.0, 0.02, ["a", "b"], cands, seed=14)
    srv = serve.Server(res, slots=4, hbm_budget=1, keep_levels=True, session_factory=StubSession,
                       deadline_s=0.03)
    qs = srv.run(trace, timeout_s=60)
    assert srv.expired == len(qs) and srv.cancelled == 0
    assert all(q.status == "expired" and q.t_done - q.t_arrival >= 0.03 for q in qs)
    st = serve.summarize(qs, res, "none")
    assert st["completed"] == 0 and "p50_ms" not in st


def test_allocation_failures_are_absorbed():
    """Sessions whose device allocation fails (ENOMEM) are retried later;
    every query is still answered exactly, and the failures are counted."""
    from paper_1708_01159_amd import gsw

    fails = {"left": 3}

    def flaky(graph, slots):
        if fails["left"] > 0:
            fails["left"] -= 1
            raise gsw.GswError(gsw.ENOMEM, "injected: hipMalloc failed")
        return StubSession(graph, slots)

    res, cands = make(["a", "b"])
    trace = serve.poisson_trace(2000.0, 0.02, ["a", "b"], cands, seed=12)
    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=flaky)
    qs = srv.run(trace, timeout_s=60)
    assert srv.alloc_failures == 3 and all(q.status == "done" for q in qs)
    for q in qs:
        g = res[q.graph].graph.csr
        assert np.array_equal(q.levels, oracle.levels(g.offs, g.cols, q.source))

    def broken(graph, slots):
        raise gsw.GswError(gsw.EINVAL, "not an allocation failure")

    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=broken)
    with pytest.raises(gsw.GswError):
        srv.run(trace[:3], timeout_s=60)


def test_lane_allocation_failure_falls_back_to_sessions():
    res, cands = make(["a"])

    def no_lane(graph):
        raise MemoryError("injected")

    trace = serve.poisson_trace(300.0, 0.03, ["a"], cands, seed=13)
    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=StubSession, solo=True, solo_factory=no_lane)
    qs = srv.run(trace, timeout_s=60)
    assert srv.alloc_failures == 1 and srv.solo_served == 0
    assert all(q.status == "done" and q.path == "session" for q in qs)


def test_worker_error_cancels_closes_and_raises():
    """A session step that fails on one graph ends the run with that error
    only after the other graphs' in-flight queries are cancelled, every worker
    has returned and every session is closed (none is left stepping)."""
    from paper_1708_01159_amd import gsw

    opened, closed = [], []

    class Tracked(SlowStubSession):
        def __init__(self, graph, slots):
            super().__init__(graph, slots)
            opened.append(self)

        def step(self, max_levels):
            if self.g.n == 600 and self.it >= 3:
                raise gsw.GswError(gsw.EHIP, "injected: level 3 finished without reporting")
            return super().step(max_levels)

        def close(self):
            closed.append(self)

    res, cands = make(["p", "a", "b"])
    trace = serve.poisson_trace(3000.0, 0.05, ["p", "a", "b"], cands, seed=14)
    srv = serve.Server(res, slots=4, keep_levels=True, session_factory=Tracked)
    with pytest.raises(gsw.GswError, match="level 3"):
        srv.run(trace, timeout_s=60)
    assert opened and sorted(map(id, closed)) == sorted(map(id, opened))
    assert not srv.sessions and not srv.workers
    assert all(f.done() for f in srv._live.values())
    for s in opened:
        assert not s.state, "a query was left running in a closed session"
