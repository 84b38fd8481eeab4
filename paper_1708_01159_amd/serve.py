"""Serving: single-source BFS queries over several resident graphs, with
continuous batching, admission by device memory, and latency percentiles.

Each graph that has queries gets a gsw session (a continuously batched
multi-source traversal with a fixed number of slots).  A query is admitted
into a free slot of its graph's session as soon as one is free -- also while
the session's other queries are mid-traversal; it joins at the next level
boundary.  Sessions are created only while their device memory (as the
library counts it, gsw_session_bytes) fits the budget; an idle session (no
slot in use) is destroyed to make room for another graph's.  A graph's
single-source lane is charged too: the graph's single-source workspace
(held until the graph is destroyed) plus the lane's level buffer, once,
when the lane is first opened.  Each session is stepped by its own worker thread on its own
HIP stream, so the work of different graphs overlaps on the device.

Optionally each graph also has a single-source lane running the
tree-switched single-source path (bitmap frontiers, the fastest way to
answer one query).  A waiting query takes the lane when it is free; the
queue goes to the session once it is long enough that waiting for the lane
one query at a time would take longer than a session query (both latencies
are tracked as moving averages per graph).  At low load queries see
single-source latency; under load the session batches them.

Latency of a query = completion time - arrival time.  Throughput = sum over
queries of the undirected edges of the source's component / makespan.

Failure handling: with a per-query deadline (seconds after arrival) a query
still waiting when it passes is dropped ("expired") and one running in a
session is cancelled ("cancelled": its slot stops at the next level boundary
and is freed without a result); a query on the single-source lane, a few
milliseconds long, always completes.  A session or lane whose device
allocation fails (ENOMEM, out of memory) is not an error: its queries keep
waiting, idle sessions of other graphs are closed to make room, and the
failure is counted.  Latency percentiles and throughput count completed
queries only; the summary gives the expired and cancelled counts beside them.

The one-at-a-time reference serves the same arrival trace in FIFO order with
one tree-switched gsw_bfs per query.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor
from concurrent.futures import wait as futures_wait
from dataclasses import dataclass, field

import numpy as np

from . import gsw


@dataclass
class Query:
    qid: int
    graph: str
    source: int
    t_arrival: float
    t_admit: float = -1.0
    t_done: float = -1.0
    levels: object = None
    path: str = ""  # "solo" or "session"
    status: str = "done"  # "done", "expired" (dropped while waiting) or "cancelled" (stopped while running)


@dataclass
class Resident:
    """A graph in device memory with what serving needs to know about it."""

    name: str
    graph: gsw.Graph
    comp_edges: np.ndarray = None  # undirected edges of the component of each vertex
    session_bytes: int = 0


def component_edges(offs, cols) -> np.ndarray:
    """Per vertex: undirected edges in its connected component (host; used to
    account throughput, not to answer queries)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    n = offs.shape[0] - 1
    a = sp.csr_matrix((np.ones(cols.shape[0], dtype=np.int8), cols, offs), shape=(n, n))
    _, lab = connected_components(a, directed=False)
    deg = np.diff(offs)
    per = np.bincount(lab, weights=deg).astype(np.int64) // 2
    return per[lab]


def session_bytes(graph, slots: int) -> int:
    """Device bytes a session of ``slots`` slots on ``graph`` allocates."""
    return graph.session_bytes(slots)


def lane_bytes(graph) -> int:
    """Device bytes of a single-source lane's level row (the graph's
    single-source workspace is charged separately, once per graph)."""
    return 4 * graph.n


def _is_oom(e: BaseException) -> bool:
    """A device allocation failure: the library's ENOMEM or torch's out-of-memory."""
    if isinstance(e, gsw.GswError):
        return e.status == gsw.ENOMEM
    return isinstance(e, MemoryError) or (isinstance(e, RuntimeError) and "out of memory" in str(e))


def poisson_trace(rate_qps: float, duration_s: float, graphs, candidates, zipf_s: float = 1.1,
                  seed: int = 107):
    """Arrival times (Poisson), graph choice Zipf(zipf_s) over ``graphs`` in the
    given order, source uniform over ``candidates[graph]``."""
    rng = np.random.default_rng(seed)
    k = len(graphs)
    p = 1.0 / np.arange(1, k + 1) ** zipf_s
    p /= p.sum()
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_qps)
        if t >= duration_s:
            break
        gi = int(rng.choice(k, p=p))
        cand = candidates[graphs[gi]]
        out.append((t, graphs[gi], int(cand[rng.integers(0, cand.shape[0])])))
    return out


class SoloLane:
    """One tree-switched single-source BFS at a time on one graph, on its own
    stream (the session of the same graph runs beside it)."""

    def __init__(self, graph: gsw.Graph, tree=None):
        import torch

        from . import trees

        self.stream = torch.cuda.Stream()
        self.levels = torch.empty((1, graph.n), dtype=torch.int32, device="cuda")
        self.runner = gsw.Runner(graph, self.levels, None, policy="tree",
                                 tree=tree if tree is not None else trees.load_default(),
                                 stream=self.stream.cuda_stream)

    def run(self, source: int, keep: bool):
        self.runner.run(int(source))
        return self.levels[0].cpu().numpy() if keep else None


class Server:
    """Continuous batching over resident graphs.

    The main loop admits arriving queries into free slots of their graph's
    session at any time; a worker thread per session keeps stepping it (the
    session takes new admissions at every level boundary inside its step),
    fetches finished slots and records their completion time.  The worker
    ends when its session has nothing admitted or running; the main loop
    starts a new one when queries are admitted again."""

    def __init__(self, residents: dict, slots: int = 64, hbm_budget: int = None,
                 levels_per_step: int = 1 << 20, keep_levels: bool = False, session_factory=None,
                 solo: bool = False, solo_factory=None, deadline_s: float = None):
        self.res = residents
        self.new_session = session_factory or gsw.Session
        self.solo = solo
        self.new_solo = solo_factory or SoloLane
        self._solo_lanes = {}       # graph -> (lane, single-thread executor)
        self._lane_failed = set()   # graphs whose lane could not be allocated (not tried again)
        self.solo_served = 0
        self.slots = slots
        self.budget = hbm_budget
        self.levels_per_step = levels_per_step
        self.keep = keep_levels
        self.sessions = {}          # graph -> gsw.Session
        self.workers = {}           # graph -> single-thread executor
        self.used = 0               # device bytes charged: open sessions, open lanes, workspaces
        self._ws_charged = set()    # graphs whose single-source workspace is charged (held for good)
        self._held = 0              # bytes lanes hold: open lanes' rows and the charged workspaces
        self.evictions = 0
        self.deadline = deadline_s  # seconds after arrival, or None
        self.expired = 0            # dropped while waiting
        self.cancelled = 0          # stopped while running in a session
        self.alloc_failures = 0     # sessions or lanes whose device allocation failed
        self._scratch_bufs = {}
        self._live = {}             # graph -> future of its running worker
        self._slot_mu = threading.Lock()

    def _ensure_session(self, name):
        if name in self.sessions:
            return self.sessions[name]
        need = session_bytes(self.res[name].graph, self.slots)
        if self.budget is not None:
            # make room by closing idle sessions of other graphs
            while self.used + need > self.budget:
                idle = [g for g, s in self.sessions.items() if s.info()["busy"] == 0 and g not in self._live]
                if not idle:
                    return None
                self._close(idle[0])
                self.evictions += 1
        try:
            s = self.new_session(self.res[name].graph, self.slots)
        except Exception as e:  # noqa: BLE001 (only allocation failures are absorbed)
            if not _is_oom(e):
                raise
            # the device is fuller than the budget says (other processes, fragmentation):
            # close an idle session of another graph and try again later
            self.alloc_failures += 1
            idle = [g for g, x in self.sessions.items() if x.info()["busy"] == 0 and g not in self._live]
            if idle:
                self._close(idle[0])
                self.evictions += 1
            return None
        self.sessions[name] = s
        self.workers[name] = ThreadPoolExecutor(max_workers=1)
        self.used += need
        return s

    def _close(self, name):
        s = self.sessions.pop(name)
        self.workers.pop(name).shutdown(wait=True)
        self.used -= session_bytes(self.res[name].graph, self.slots)
        s.close()

    def _scratch(self, name):
        buf = self._scratch_bufs.get(name)
        if buf is None:
            import torch

            buf = torch.empty(self.res[name].graph.n, dtype=torch.int32, device="cuda")
            self._scratch_bufs[name] = buf
        return buf

    def _work(self, name, sess, slot_q, done_q, t0):
        """Worker: step until nothing is admitted or running; each finished
        slot is fetched (which frees it) after its query has been taken off
        the slot map, so a new admission into that slot cannot be mistaken
        for it."""
        while True:
            fin, run = sess.step(self.levels_per_step)
            for k in fin:
                with self._slot_mu:
                    q = slot_q.pop(k)
                out = np.empty(self.res[name].graph.n, dtype=np.int32) if self.keep else self._scratch(name)
                sess.fetch(k, out)
                q.t_done = time.perf_counter() - t0
                q.levels = out if self.keep else None
                q.path = "session"
                done_q.append(q)
            if run == 0 and not fin:
                return

    def _solo_run(self, name, lane, q, done_q, t0):
        q.levels = lane.run(q.source, self.keep)
        q.t_done = time.perf_counter() - t0
        q.path = "solo"
        done_q.append(q)

    def _solo_lane(self, name):
        """The graph's single-source lane, opened (and charged) on first use;
        None when the budget has no room for it (its queries then go to the
        session)."""
        if name in self._lane_failed:
            return None
        if name not in self._solo_lanes:
            g = self.res[name].graph
            need = lane_bytes(g) + (0 if name in self._ws_charged else g.workspace_bytes())
            if self.budget is not None:
                # lanes hold their bytes for the rest of the run (workspaces for
                # good): open one only while the largest session still fits
                # beside everything lanes hold, so no graph's queries can be
                # locked out of a session
                biggest = max(session_bytes(r.graph, self.slots) for r in self.res.values())
                if self._held + need + biggest > self.budget:
                    return None
            try:
                lane = self.new_solo(g)
            except Exception as e:  # noqa: BLE001
                if not _is_oom(e):
                    raise
                self.alloc_failures += 1
                self._lane_failed.add(name)
                return None
            self._solo_lanes[name] = (lane, ThreadPoolExecutor(max_workers=1))
            self.used += need
            self._held += need
            self._ws_charged.add(name)
        return self._solo_lanes[name]

    def _expire(self, pending, slot_q, now):
        """Deadline pass: drops waiting queries past their deadline and cancels
        those running in a session; returns how many ended here."""
        ended = 0
        for dq in pending.values():
            while dq and now - dq[0].t_arrival > self.deadline:  # FIFO: oldest first
                q = dq.popleft()
                q.status, q.t_done = "expired", now
                self.expired += 1
                ended += 1
        for name, slots in slot_q.items():
            sess = self.sessions.get(name)
            for k, q in list(slots.items()):
                if now - q.t_arrival <= self.deadline or sess is None:
                    continue
                with self._slot_mu:  # a worker takes finished slots off the map under the same lock
                    if slots.get(k) is q and sess.cancel(k):
                        del slots[k]
                        q.status, q.t_done = "cancelled", now
                        self.cancelled += 1
                        ended += 1
        return ended

    def run(self, trace, timeout_s: float = 600.0):
        """Serves ``trace`` = [(t_arrival, graph, source)] in real time; returns
        the list of completed Query objects.  On an error (a worker's, or the
        time limit) every query still in a slot is cancelled, the workers are
        waited for and the sessions closed before the error is raised."""
        self._slot_q = collections.defaultdict(dict)  # graph -> slot -> Query (admitted, not yet fetched)
        self._live = {}                               # graph -> worker future
        self._solo_busy = {}                          # graph -> future of its single-source lane
        try:
            queries = self._serve(trace, timeout_s)
        except BaseException:
            self._abandon()
            raise
        self._shut()
        return queries

    def _abandon(self):
        with self._slot_mu:
            for name, slots in self._slot_q.items():
                sess = self.sessions.get(name)
                for k in list(slots):
                    if sess is not None and sess.cancel(k):
                        del slots[k]
        for fut in list(self._live.values()) + list(self._solo_busy.values()):
            try:
                fut.result()
            except Exception:  # noqa: BLE001 (the first error is the one raised)
                pass
        self._shut()

    def _shut(self):
        for name in list(self.sessions):
            self._close(name)
        for name, (lane, ex) in self._solo_lanes.items():
            ex.shutdown(wait=True)
            self.used -= lane_bytes(self.res[name].graph)
            self._held -= lane_bytes(self.res[name].graph)
        self._solo_lanes = {}

    def _serve(self, trace, timeout_s):
        queries = [Query(i, g, s, t) for i, (t, g, s) in enumerate(sorted(trace))]
        pending = collections.defaultdict(collections.deque)
        slot_q = self._slot_q
        done_q = collections.deque()            # completed queries, appended by workers
        solo_busy = self._solo_busy
        est = collections.defaultdict(lambda: {"solo": 0.5e-3, "session": 1.0e-3})  # s, moving averages
        nxt = 0
        done = 0
        t0 = time.perf_counter()
        while done < len(queries):
            now = time.perf_counter() - t0
            if now > timeout_s:
                raise TimeoutError("serving run exceeded %.0f s: %d of %d done, %d waiting, %d in slots" % (
                    timeout_s, done, len(queries), sum(map(len, pending.values())),
                    sum(map(len, slot_q.values()))))
            while nxt < len(queries) and queries[nxt].t_arrival <= now:
                pending[queries[nxt].graph].append(queries[nxt])
                nxt += 1
            while done_q:
                q = done_q.popleft()
                e = est[q.graph]
                e[q.path] = 0.8 * e[q.path] + 0.2 * (q.t_done - q.t_admit)
                done += 1
            if self.deadline is not None:
                done += self._expire(pending, slot_q, now)
            for name, fut in list(self._live.items()):
                if fut.done():
                    del self._live[name]
                    fut.result()  # re-raises a worker's error
            for name, fut in list(solo_busy.items()):
                if fut.done():
                    del solo_busy[name]
                    fut.result()
            # admission: the single-source lane when the graph has nothing in
            # flight, else free slots of the graph's session (created under the budget)
            for name, dq in pending.items():
                if not dq:
                    continue
                lane = self._solo_lane(name) if self.solo else None
                if lane is not None:
                    if name not in solo_busy:
                        q = dq.popleft()
                        q.t_admit = time.perf_counter() - t0
                        solo_busy[name] = lane[1].submit(self._solo_run, name, lane[0], q, done_q, t0)
                        self.solo_served += 1
                    # the rest waits for the lane unless the session would be quicker
                    e = est[name]
                    if not dq or len(dq) * e["solo"] < e["session"]:
                        continue
                sess = self._ensure_session(name)
                if sess is None:
                    continue
                while dq:
                    with self._slot_mu:  # the worker may finish the slot as soon as it is admitted
                        k = sess.admit(dq[0].source)
                        if k is None:
                            break
                        q = dq.popleft()
                        q.t_admit = time.perf_counter() - t0
                        slot_q[name][k] = q
            # a worker for every session with admitted queries and none running
            for name, sess in list(self.sessions.items()):
                if name not in self._live and slot_q[name]:
                    self._live[name] = self.workers[name].submit(self._work, name, sess, slot_q[name], done_q, t0)
            if not done_q:
                until_next = queries[nxt].t_arrival - now if nxt < len(queries) else 0.001
                busy = list(self._live.values()) + list(solo_busy.values())
                if busy:
                    futures_wait(busy, timeout=max(0.0, min(until_next, 0.0002)), return_when=FIRST_COMPLETED)
                elif nxt < len(queries):
                    time.sleep(max(0.0, min(until_next, 0.001)))
        for fut in list(self._live.values()) + list(solo_busy.values()):
            fut.result()
        return queries


def serve_one_at_a_time(residents: dict, trace, tree, timeout_s: float = 600.0):
    """FIFO, one tree-switched gsw_bfs per query, in real time."""
    import torch

    queries = [Query(i, g, s, t) for i, (t, g, s) in enumerate(sorted(trace))]
    runners = {}
    for name, r in residents.items():
        lv = torch.empty((1, r.graph.n), dtype=torch.int32, device="cuda")
        runners[name] = gsw.Runner(r.graph, lv, None, policy="tree", tree=tree)
    t0 = time.perf_counter()
    for q in queries:
        now = time.perf_counter() - t0
        if now > timeout_s:
            raise TimeoutError("one-at-a-time run exceeded %.0f s" % timeout_s)
        if q.t_arrival > now:
            time.sleep(q.t_arrival - now)
        q.t_admit = time.perf_counter() - t0
        runners[q.graph].run(q.source)
        q.t_done = time.perf_counter() - t0
    return queries


def summarize(queries, residents, label):
    """Latency percentiles and throughput over the completed queries; counts of
    the expired and cancelled ones."""
    ok = [q for q in queries if q.status == "done"]
    out = {"mode": label, "queries": len(queries), "completed": len(ok),
           "expired": sum(q.status == "expired" for q in queries),
           "cancelled": sum(q.status == "cancelled" for q in queries)}
    if not ok:
        return out
    lat = np.array([q.t_done - q.t_arrival for q in ok]) * 1e3
    span = max(q.t_done for q in ok) - min(q.t_arrival for q in ok)
    edges = sum(int(residents[q.graph].comp_edges[q.source]) for q in ok)
    out.update({"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "gteps": round(edges / span / 1e9, 3),
                "makespan_s": round(span, 3)})
    return out


def per_graph_p99(queries):
    """p99 latency (ms) of each graph's completed queries."""
    by = {}
    for q in queries:
        if q.status != "done":
            continue
        by.setdefault(q.graph, []).append((q.t_done - q.t_arrival) * 1e3)
    return {g: round(float(np.percentile(v, 99)), 3) for g, v in sorted(by.items())}
