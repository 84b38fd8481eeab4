#!/usr/bin/env python3
"""Benchmark: GTEPS of tree-switched BFS on R-MAT scale 22 vs every fixed
kernel and the best-per-level schedule, on one MI355X; batched multi-source
BFS; the structure sweep; and continuous-batching serving with p50/p99.

One step = a tree-switched BFS (level loop, per-level kernel choice, every
expansion kernel it picks) from each of the 64 seeded sources of the
workload.  GTEPS of a source = undirected edges of its component / time of
its gsw_bfs call (graph upload and result copy-back excluded, as in the
paper's measurements); the reported value is the harmonic mean over sources
of each source's median over the timed steps.

Prints ONE JSON line.  Besides the contract fields:
  fixed            harmonic-mean GTEPS of each of the 33 kernels (11 base
                   kernels x 3 frontier-count variants) used at every level
  best_per_level   GTEPS of replaying, per source (all 64), the fastest kernel
                   of each level (times measured from the same saved state)
  tree_agreement   share of levels where the tree picked that fastest kernel
  roofline         the dominant kernel of the switched path: algorithmic bytes
                   per launch (mean over every launch of that kernel in an
                   instrumented pass over all 64 sources, right after the
                   timed steps) / its mean launch time in that pass, timed
                   with HIP events recorded on the search's stream after
                   every launch; both byte models are given (the library's
                   model and the scope table's literal pull formula);
                   traffic = HBM bytes per launch from the committed
                   rocprofv3 counter summary while the kernel source it was
                   taken on is unchanged, with that summary's mean kernel
                   duration and the fraction it gives (the event brackets
                   also hold the gap before each launch starts)
  cpu_baseline     the CPU oracle on a bounded sample of the same sources
  batched          R-MAT scale 20, B = 64/256/1024 vs the same sources one at a
                   time; thresholds and block size tuned on a disjoint sample
  sweep            grid 2048^2 (5% deleted), Chung-Lu 2^23, Erdos-Renyi 2^22
  serving          eight resident graphs, Poisson arrivals at 100-5000 QPS

A time guard (--budget, default 540 s) skips the remaining optional
sections, saying so in the line, when the run is late.

Profiling: every expansion variant runs inside one kernel (k_level_auto),
so rocprofv3's per-kernel view cannot tell them apart.  ``--dispatch-log``
records, for every BFS call, each level's kernel, frontier and algorithmic
bytes; ``--summarize-profile DIR`` (no GPU) aligns the per-dispatch rows of
the kernel trace and of the FETCH_SIZE / WRITE_SIZE counter runs in DIR with
that log and prints the per-variant summary kept under profiles/
(paper_1708_01159_amd/profile_summary.py).  ``--batched-only 1024`` runs
only the batched section.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS (RMAT-22) switched vs best fixed kernel; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {
    "rmat22": "R-MAT scale 22 (4,194,304 vertices), edgefactor 16, A/B/C/D .57/.19/.19/.05, "
              "seed 2, symmetrised, loops and repeats removed, int32 CSR with int64 offsets; "
              "64 seeded sources of degree > 0",
}
T0 = time.perf_counter()


def log(*a):
    print("[bench %6.1fs]" % (time.perf_counter() - T0), *a, file=sys.stderr, flush=True)


def hmean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(len(x) / np.sum(1.0 / x)) if len(x) else 0.0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, srcs, m_c, budget_s):
    """The CPU oracle (single thread) on as many sources as fit in budget_s."""
    import oracle  # test infrastructure, used only for this reported baseline

    times, edges = [], []
    t_start = time.perf_counter()
    for i, s in enumerate(srcs):
        t0 = time.perf_counter()
        oracle.levels(g.offs, g.cols, int(s))
        times.append(time.perf_counter() - t0)
        edges.append(m_c[i])
        if time.perf_counter() - t_start > budget_s:
            break
    gteps = [e / t / 1e9 for e, t in zip(edges, times)]
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"value": round(hmean(gteps), 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "%d of %d sources of the same workload, single-threaded FIFO BFS, %.1f s"
                      % (len(times), len(srcs), sum(times)),
            "cpu": cpu_model(), "host_nproc": os.cpu_count(), "host_cpus_available": affinity}


def committed_profile(kernel_name):
    """Fields of the committed rocprofv3 summary of ``kernel_name`` (HBM
    traffic per launch, mean duration, dispatches), or None when that summary
    is missing, is for another kernel, or was taken on a different kernel
    source."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_rmat22.md" % kernel_name)
    src = os.path.join(ROOT, "paper_1708_01159_amd", "csrc", "gsw_kernels.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    keys = ("traffic_bytes_per_launch", "kernel", "kernel_source_sha256", "mean_duration_us", "dispatches",
            "algorithmic_bytes_per_launch")
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and line.split(": ", 1)[0] in keys)
    if fields.get("kernel") != kernel_name or fields.get("kernel_source_sha256") != sha:
        return None
    return fields


def copy_calibration():
    """A plain 1 GiB device copy (torch), twice: the profiler's counters for
    it scale the counter runs of the same command."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    ev0.record()
    b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    out = {"bytes_read": a.numel() * 4, "bytes_written": a.numel() * 4, "ms": round(ms, 4),
           "gbs": round(2 * a.numel() * 4 / ms / 1e6, 1)}
    del a, b
    return out


def timed(runner, src, sync):
    sync()
    t0 = time.perf_counter()
    runner.run(int(src))
    return time.perf_counter() - t0


def _logged(runner, tag, calls, counts=None, src_index=None):
    """Runner whose every call appends its levels' (kernel, frontier, bytes)
    to calls."""
    if calls is None:
        return runner
    from paper_1708_01159_amd import traffic

    run = runner.run

    def logged_run(source):
        nrows = run(source)
        c = counts.get(int(source)) if counts is not None else None
        lv = []
        for r in runner.rows():
            b = traffic.level_bytes(r.kernel, c, r.level) if c is not None else None
            lit = traffic.pull_bytes_literal(c, r.level) if c is not None and r.kernel % 11 == 7 else None
            lv.append([r.kernel, r.n_frontier, b, lit, r.launch, r.flags])
        calls.append({"tag": tag, "source": int(source), "levels": lv})
        return nrows

    runner.run = logged_run
    return runner


# --------------------------------------------------------------- headline
def run_headline(args, g, G, tree, srcs, calls):
    """Timed steps of the switched path, the instrumented pass, the roofline."""
    import torch

    from paper_1708_01159_amd import gsw, traffic

    sync = torch.cuda.synchronize
    n = g.n
    out_lv = torch.empty((1, n), dtype=torch.int32, device="cuda")
    out_pa = torch.empty((1, n), dtype=torch.int32, device="cuda")
    deg = g.degrees()
    counts = {}
    sw = _logged(gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree), "switched", calls, counts)
    # the same path with a HIP event after every launch (kept out of the timed steps)
    sw_ev = _logged(gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree, time_levels=2), "event-timed levels",
                    calls, counts)
    m_c = np.zeros(len(srcs), dtype=np.int64)
    for w in range(max(args.warmup, 1)):
        for i, s in enumerate(srcs):
            sw.run(int(s))
            if w == 0:
                lv = out_lv[0].cpu().numpy()
                m_c[i] = int(deg[lv >= 0].sum() // 2)
                counts[int(s)] = traffic.Counts(g.offs, g.cols, lv, int(s))
    log("warm-up done (%d sources, byte-model counts taken)" % len(srcs))
    per_src = np.zeros((args.steps, len(srcs)))
    sync()
    t_all = time.perf_counter()
    for k in range(args.steps):
        for i, s in enumerate(srcs):
            per_src[k, i] = timed(sw, s, sync)
    sync()
    wall = time.perf_counter() - t_all
    med = np.median(per_src, axis=0)
    gteps_src = m_c / med / 1e9
    value = hmean(gteps_src)
    log("switched: %.2f GTEPS (harmonic), %.2f ms/step, %.3f ms median source"
        % (value, wall / args.steps * 1e3, np.median(med) * 1e3))
    # instrumented pass: per-level times from HIP events around every launch
    traces, per_src_ev = [], np.zeros(len(srcs))
    for i, s in enumerate(srcs):
        per_src_ev[i] = timed(sw_ev, s, sync)
        traces.append((i, int(s), sw_ev.rows()))
    nk = gsw.N_KERNELS
    ktime = np.zeros(nk)
    kcount = np.zeros(nk, dtype=np.int64)
    for _, _, tr in traces:
        for r in tr:
            ktime[r.kernel] += r.ms
            kcount[r.kernel] += 1
    dom = int(np.argmax(ktime))
    b_model, b_lit, t_sum, launches = 0, 0, 0.0, 0
    for _, s, tr in traces:
        c = counts[s]
        for r in tr:
            if r.kernel == dom:
                b_model += traffic.level_bytes(dom, c, r.level)
                if dom % 11 == traffic.PULL:
                    b_lit += traffic.pull_bytes_literal(c, r.level)
                t_sum += r.ms * 1e-3
                launches += 1
    mean_b = b_model / max(launches, 1)
    mean_t = t_sum / max(launches, 1)
    achieved = mean_b / mean_t / 1e9 if mean_t > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": gsw.KERNEL_NAMES[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None,
                "bytes_per_launch": int(round(mean_b)),
                "mean_launch_ms": round(mean_t * 1e3, 5),
                "launches": launches, "sources": len(srcs),
                "timing": "HIP events recorded on the search's stream after every launch",
                "share_of_kernel_time": round(float(ktime[dom] / ktime.sum()), 3)}
    prof = committed_profile(gsw.KERNEL_NAMES[dom])
    if prof:
        # the rocprofv3 kernel trace of the profiling command: its mean
        # duration excludes the dispatch gap that the event brackets include
        roofline["traffic"] = int(prof["traffic_bytes_per_launch"])
        d_us = float(prof["mean_duration_us"])
        roofline["rocprof_mean_launch_us"] = d_us
        roofline["rocprof_dispatches"] = int(prof["dispatches"])
        roofline["frac_rocprof_duration"] = round(mean_b / (d_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    if b_lit:
        lit = b_lit / launches
        roofline["bytes_per_launch_literal"] = int(round(lit))
        roofline["frac_literal"] = round(lit / mean_t / 1e9 / HBM_PEAK_GBS, 4)
    roofline["instrumented_pass_median_source_ms"] = round(float(np.median(per_src_ev)) * 1e3, 4)
    log("roofline %s: %.1f MB/launch over %d launches, %.2f us -> %.0f GB/s (%.3f of peak)"
        % (gsw.KERNEL_NAMES[dom], mean_b / 1e6, launches, mean_t * 1e6, achieved, achieved / HBM_PEAK_GBS))
    shares = {gsw.KERNEL_NAMES[k]: round(float(ktime[k] / ktime.sum()), 3) for k in range(nk) if kcount[k]}
    return dict(value=value, wall=wall, med=med, gteps_src=gteps_src, m_c=m_c, traces=traces, roofline=roofline,
                shares=shares, kernel_ms=float(ktime.sum() / len(srcs)), out_lv=out_lv, out_pa=out_pa, counts=counts)


def run_fixed(G, srcs, m_c, out_lv, out_pa, kernels=None):
    import torch

    from paper_1708_01159_amd import gsw

    sync = torch.cuda.synchronize
    fixed = {}
    for kern in (kernels if kernels is not None else range(gsw.N_KERNELS)):
        fx = gsw.Runner(G, out_lv, out_pa, policy="fixed", kernel=kern, trace_cap=1 << 16)
        fx.run(int(srcs[0]))  # warm
        ts = np.array([timed(fx, s, sync) for s in srcs])
        fixed[gsw.KERNEL_NAMES[kern]] = round(hmean(m_c / ts / 1e9), 3)
    return fixed


def level_times(G, s, reps):
    """Per-level time (ms) of every kernel from the same saved state
    (gsw_bfs_profile), with the push kernels' times on the levels the search
    runs in single-workgroup multi-level launches replaced by what such a
    launch costs per level -- the correction the tree's training rows get
    (paper_1708_01159_amd.train.apply_solo): the profile times each level as
    a launch of its own."""
    from paper_1708_01159_amd import gsw, train

    times, fr, ks = gsw.bfs_profile(G, int(s), reps=reps, advance_kernel=-1)
    _, _, tr = gsw.bfs(G, [int(s)], policy="fixed", kernel=gsw.PUSH_VERTEX, parents=False, time_levels=True,
                       trace_cap=len(fr) + 64)
    solo = np.full(len(fr), np.nan)
    for t in tr:
        if t.level < len(fr) and t.flags & 4:
            solo[t.level] = t.ms
    return train.apply_solo(times, solo, ks)


def run_best_per_level(G, srcs, m_c, med_switched, traces, out_lv, out_pa, reps, steps):
    """Per source: each level's fastest kernel measured from the same saved
    state (all 33 kernels; level_times), replayed end to end."""
    import torch

    from paper_1708_01159_amd import gsw

    sync = torch.cuda.synchronize
    t_bpl, agree, levels_total, regret = [], 0, 0, 0.0
    sched_runner = gsw.Runner(G, out_lv, out_pa, policy="schedule", schedule=[0], trace_cap=1 << 16)
    picks_of = {i: [r.kernel for r in tr] for i, _, tr in traces}
    for i, s in enumerate(srcs):
        times = level_times(G, s, reps)
        sched = np.argmin(times, axis=1).astype(np.int32)
        sched_runner.set_schedule(sched)
        sched_runner.run(int(s))
        t_bpl.append(np.median([timed(sched_runner, s, sync) for _ in range(max(steps, 1))]))
        for d, kk in enumerate(picks_of.get(i, [])[:len(sched)]):
            agree += int(kk == sched[d])
            regret += float(times[d, kk] - times[d, sched[d]])
            levels_total += 1
    t_bpl = np.array(t_bpl)
    return {"gteps": round(hmean(m_c / t_bpl / 1e9), 3), "sources": len(srcs), "kernels": gsw.N_KERNELS,
            "profile_reps": reps,
            "switched_time_over_best_per_level": round(float(np.sum(med_switched) / t_bpl.sum()), 4),
            "per_source_ratio_median": round(float(np.median(med_switched / t_bpl)), 4),
            "tree_agreement": {"levels": levels_total, "fastest_picked": round(agree / max(levels_total, 1), 3),
                               "mean_regret_ms_per_source": round(regret / len(srcs), 4)}}


# ---------------------------------------------------------------- batched
def bench_batched(batches=(64, 256, 1024)):
    """Batched multi-source BFS on R-MAT scale 20 vs the same sources one at a
    time on the tree-switched single-source path.  The thresholds and the
    block size are tuned on another batch of the same size (sources from a
    different seed), then the timed batch runs with them."""
    import torch

    from paper_1708_01159_amd import autotune, gsw, serve, trees
    from paper_1708_01159_amd import graphgen as gg

    sync = torch.cuda.synchronize
    g = gg.workload("rmat20")
    k, seed = gg.WORKLOAD_SOURCES["rmat20"]
    srcs = gg.pick_sources(g, max(batches), seed)
    tune_srcs = gg.pick_sources(g, max(batches), seed + 100)
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    ce = serve.component_edges(g.offs, g.cols)
    tree = trees.load_default()
    lv1 = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
    single = gsw.Runner(G, lv1, None, policy="tree", tree=tree)
    single.run(int(srcs[0]))
    t_single = np.array([timed(single, s, sync) for s in srcs])
    out = {}
    for B in batches:
        src = srcs[:B]
        p2p, p2s, bs, table = autotune.tune(G, tune_srcs[:B])
        lvB = torch.empty((B, g.n), dtype=torch.int8, device="cuda")
        gsw.msbfs(G, src, p2p, p2s, out=lvB, block_size=bs)
        ts = []
        for _ in range(5):
            sync()
            t0 = time.perf_counter()
            _, nl = gsw.msbfs(G, src, p2p, p2s, out=lvB, block_size=bs)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        edges = int(ce[src].sum())
        one = float(t_single[:B].sum())
        out[str(B)] = {"ms": round(t * 1e3, 3), "gteps": round(edges / t / 1e9, 2),
                       "push_to_pull": p2p, "pull_to_push": p2s, "block_size": bs,
                       "one_at_a_time_ms": round(one * 1e3, 3),
                       "one_at_a_time_gteps": round(edges / one / 1e9, 2),
                       "speedup": round(one / t, 2), "levels": nl}
        log("batched B=%d: %.2f ms (%.1f GTEPS) vs one at a time %.2f ms (%.1f GTEPS); thresholds %g/%g, block %d"
            % (B, t * 1e3, edges / t / 1e9, one * 1e3, edges / one / 1e9, p2p, p2s, bs))
    G.close()
    return {"workload": "R-MAT scale 20 (1,048,576 vertices), edgefactor 16, seed 6; timed sources seed 106",
            "level_type": "int8",
            "tuning": "thresholds and block size tuned per batch size on sources of seed 206 (disjoint sample)",
            "batches": out}


# ------------------------------------------------------------------ sweep
SWEEP = (("grid2048_del5", 1, 1), ("chunglu23", 8, 2), ("er22", 8, 2))  # (graph, best-per-level sources, reps)


def bench_sweep(tree):
    """Structure sweep: switched vs every fixed kernel (all 32 sources) vs
    best-per-level (the stated sample of sources)."""
    import torch

    from paper_1708_01159_amd import gsw
    from paper_1708_01159_amd import graphgen as gg

    sync = torch.cuda.synchronize
    res = {}
    graphs = {}
    for name, bpl_src, reps in SWEEP:
        t = time.perf_counter()
        g = gg.workload(name)
        graphs[name] = g
        k, seed = gg.WORKLOAD_SOURCES[name]
        srcs = gg.pick_sources(g, k, seed)
        G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
        lv = torch.empty((1, g.n), dtype=torch.int32, device="cuda")
        deg = g.degrees()
        sw = gsw.Runner(G, lv, None, policy="tree", tree=tree, trace_cap=1 << 16)
        m_c = np.zeros(len(srcs), dtype=np.int64)
        for i, s in enumerate(srcs):
            sw.run(int(s))
            m_c[i] = int(deg[lv[0].cpu().numpy() >= 0].sum() // 2)
        t_sw = np.array([min(timed(sw, s, sync), timed(sw, s, sync)) for s in srcs])
        fixed = run_fixed(G, srcs, m_c, lv, None)
        bf = max(fixed, key=fixed.get)
        sched = gsw.Runner(G, lv, None, policy="schedule", schedule=[0], trace_cap=1 << 16)
        r_sw, r_bpl = [], []
        for i, s in enumerate(srcs[:bpl_src]):
            times = level_times(G, s, reps)
            sched.set_schedule(np.argmin(times, axis=1).astype(np.int32))
            sched.run(int(s))
            r_bpl.append(min(timed(sched, s, sync), timed(sched, s, sync)))
            r_sw.append(t_sw[i])
        gt = hmean(m_c / t_sw / 1e9)
        res[name] = {"n": g.n, "nnz": g.nnz, "sources": len(srcs), "switched_gteps": round(gt, 3),
                     "fixed": fixed, "best_fixed": bf, "switched_over_best_fixed": round(gt / fixed[bf], 3),
                     "switched_time_over_best_per_level": round(float(np.sum(r_sw) / np.sum(r_bpl)), 4),
                     "best_per_level_sources": bpl_src, "best_per_level_profile_reps": reps}
        log("sweep %s: switched %.3f GTEPS, best fixed %s %.3f, vs best-per-level %.3f (%.0f s)"
            % (name, gt, bf, fixed[bf], res[name]["switched_time_over_best_per_level"], time.perf_counter() - t))
        G.close()
    return res, graphs


# ----------------------------------------------------- connected components
def bench_components(tree, preloaded):
    """Weakly connected components (gsw_cc) on the headline graph and the
    sweep's scale-free graph: the default path (the tree-switched BFS for the
    largest-degree component, then propagation with push or pull chosen per
    iteration) and propagation alone under each policy, against the oracle's
    result and time; the pull kernel's algorithmic bytes per iteration."""
    import torch

    import oracle
    from paper_1708_01159_amd import gsw

    sync = torch.cuda.synchronize
    res = {}
    for name, (g, G) in preloaded.items():
        t = time.perf_counter()
        want, count = oracle.components(g.offs, g.cols)
        t_cpu = time.perf_counter() - t
        out = torch.empty(g.n, dtype=torch.int32, device="cuda")
        row = {"n": g.n, "nnz": g.nnz, "components": count, "oracle_s": round(t_cpu, 3)}
        for label, kw in (("bfs_then_switch", dict(policy="switch")),
                          ("propagation_switch", dict(policy="switch", bfs_first=False)),
                          ("propagation_push", dict(policy="push", bfs_first=False)),
                          ("propagation_pull", dict(policy="pull", bfs_first=False))):
            best, tr = 1e9, None
            for _ in range(3):
                sync()
                t0 = time.perf_counter()
                _, nc, tr = gsw.components(G, tree=tree, device=True, out=out, **kw)
                sync()
                best = min(best, time.perf_counter() - t0)
            ok = nc == count and np.array_equal(out.cpu().numpy(), want)
            row[label] = {"ms": round(best * 1e3, 3), "iterations": len(tr), "equal_to_oracle": bool(ok),
                          "kernels": [r["kernel"] for r in tr][:16]}
            if label == "propagation_pull":
                # per pull iteration: every remaining vertex's row bounds (2 x 8 B), its label
                # and list entry (4 + 4 B), and per arc a column and a label (4 + 4 B)
                its = [r for r in tr if r["kernel"] == "pull"]
                n_rest, e_rest = tr[0]["n_active"], tr[0]["e_active"]
                b = 24 * n_rest + 8 * e_rest
                ms = float(np.mean([r["ms"] for r in its]))
                row["pull_roofline"] = {"bound": "hbm", "bytes_per_iteration": int(b), "mean_iteration_ms": round(ms, 4),
                                        "achieved_gbs": round(b / ms / 1e6, 1),
                                        "frac": round(b / ms / 1e6 / 8000.0, 4),
                                        "timing": "HIP events around each iteration"}
        row["speedup_over_oracle"] = round(t_cpu / (row["bfs_then_switch"]["ms"] * 1e-3), 1)
        log("components %s: %d components, %.3f ms (bfs then switch) vs oracle %.2f s; propagation alone "
            "switch/push/pull %.2f / %.2f / %.2f ms" % (
                name, count, row["bfs_then_switch"]["ms"], t_cpu, row["propagation_switch"]["ms"],
                row["propagation_push"]["ms"], row["propagation_pull"]["ms"]))
        res[name] = row
    return res


def components_pull_only(calls: int = 4):
    """Connected components of R-MAT 22 by propagation alone with the pull
    kernel at every iteration (each iteration reads every arc: the kernel's
    byte model is exact per launch), for the profiler: one untimed call, then
    `calls` calls; labels checked against the oracle."""
    import torch

    import oracle
    from paper_1708_01159_amd import gsw
    from paper_1708_01159_amd import graphgen as gg

    g = gg.workload("rmat22")
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    want, count = oracle.components(g.offs, g.cols)
    tr = None
    for _ in range(calls + 1):
        _, nc, tr = gsw.components(G, policy="pull", bfs_first=False, device=True, out=out)
    torch.cuda.synchronize()
    ok = nc == count and np.array_equal(out.cpu().numpy(), want)
    n_rest, e_rest = tr[0]["n_active"], tr[0]["e_active"]
    G.close()
    return {"workload": "R-MAT scale 22, seed 2", "calls": calls + 1, "iterations_per_call": len(tr),
            "n_rest": int(n_rest), "e_rest": int(e_rest), "bytes_per_iteration": int(24 * n_rest + 8 * e_rest),
            "mean_iteration_ms_events": round(float(np.mean([r["ms"] for r in tr])), 4), "equal_to_oracle": bool(ok)}


# ---------------------------------------------------------------- serving
SERVING_RATES = (100, 500, 1000, 2000, 5000)
SERVING_SECONDS = 4.0
SERVING_BUDGET = 32 << 30


def bench_serving(tree, preloaded):
    """Continuous-batching serving over eight resident graphs vs one query at
    a time, p50/p99 latency (arrival to result ready) and aggregate GTEPS."""
    from paper_1708_01159_amd import gsw, serve
    from paper_1708_01159_amd import graphgen as gg

    specs = [("rmat16", lambda: gg.rmat(16, 16, seed=7)), ("rmat18", lambda: gg.rmat(18, 16, seed=8)),
             ("rmat20", lambda: gg.rmat(20, 16, seed=9)), ("rmat22", None),
             ("rmat24", lambda: gg.rmat(24, 16, seed=11)), ("grid4096", lambda: gg.grid(4096, 4096, 0.0, seed=12)),
             ("chunglu23", None), ("er24", lambda: gg.erdos_renyi(1 << 24, 4 << 24, seed=14))]
    residents, cands = {}, {}
    t = time.perf_counter()
    for name, make in specs:
        if make is None:
            g, G = preloaded[name]
        else:
            g = make()
            G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
        residents[name] = serve.Resident(name, G, serve.component_edges(g.offs, g.cols))
        cands[name] = np.flatnonzero(g.degrees() > 0)
    log("serving: 8 graphs resident (%.0f s)" % (time.perf_counter() - t))
    names = [s[0] for s in specs]
    runs = []
    fmt = lambda r: "p50 %.2f p99 %.2f ms %.1f GTEPS" % (r["p50_ms"], r["p99_ms"], r["gteps"])
    for rate in SERVING_RATES:
        trace = serve.poisson_trace(rate, SERVING_SECONDS, names, cands, seed=107 + rate)
        row = {"rate_qps": rate, "queries": len(trace)}
        srv = serve.Server(residents, slots=64, hbm_budget=SERVING_BUDGET, solo=True)
        try:
            qb = srv.run(trace, timeout_s=150)
            row["batched"] = serve.summarize(qb, residents, "continuous batching + single-source lane")
            row["batched"]["solo_served"] = srv.solo_served
            row["batched"]["per_graph_p99_ms"] = serve.per_graph_p99(qb)
        except TimeoutError as e:
            row["batched"] = {"timed_out": str(e)}
        except gsw.GswError as e:  # recorded; the server has closed its sessions
            import traceback

            traceback.print_exc(file=sys.stderr)
            row["batched"] = {"error": str(e)}
        log("serving %d QPS batched: %s" % (rate, fmt(row["batched"]) if "p50_ms" in row["batched"] else
                                            "failed: %s" % next(iter(row["batched"].values()))))
        if rate <= 500:
            try:
                qo = serve.serve_one_at_a_time(residents, trace, tree, timeout_s=150)
                row["one_at_a_time"] = serve.summarize(qo, residents, "one at a time")
            except TimeoutError as e:
                row["one_at_a_time"] = {"timed_out": str(e)}
            log("serving %d QPS one at a time: %s" % (rate, fmt(row["one_at_a_time"])
                                                      if "p50_ms" in row["one_at_a_time"] else "timed out"))
        runs.append(row)
    for name, r in residents.items():
        if name not in preloaded:
            r.graph.close()
    return {"graphs": names, "zipf": 1.1, "duration_s_per_rate": SERVING_SECONDS, "slots": 64,
            "hbm_budget_bytes": SERVING_BUDGET,
            "note": "rmat22 is the headline graph (seed 2) and chunglu23 the sweep's (seed 4); the others use "
                    "seeds 7-14; one at a time is run up to 500 QPS (it saturates beyond)",
            "runs": runs}


def optional_section(name, fn, *a):
    """Runs one of the comparison sections after the headline; a library error
    there is recorded in the JSON line (with its traceback on stderr) instead
    of ending the run before the headline is printed."""
    from paper_1708_01159_amd import gsw

    try:
        return fn(*a)
    except (gsw.GswError, TimeoutError) as e:
        import traceback

        traceback.print_exc(file=sys.stderr)
        log("%s section failed: %s" % (name, e))
        return {"error": "%s: %s" % (type(e).__name__, e)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=None, help="override the source count")
    ap.add_argument("--tree", default=None, help="tree JSON (default: shipped tree)")
    ap.add_argument("--no-compare", action="store_true",
                    help="only the timed switched path and its instrumented pass (for profiling runs)")
    ap.add_argument("--profile-reps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--budget", type=float, default=540.0, help="seconds after which optional sections are skipped")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-components", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    ap.add_argument("--dispatch-log", default=None,
                    help="write every BFS call's (kernel, frontier, bytes) per level to this JSON file")
    ap.add_argument("--batched-only", default=None, metavar="B[,B...]",
                    help="only the batched section at these batch sizes (one JSON line; for profiling)")
    ap.add_argument("--components-only", action="store_true",
                    help="only connected components on R-MAT 22 by pull propagation (one JSON line; for profiling)")
    ap.add_argument("--summarize-components", default=None, metavar="DIR",
                    help="print the components rocprofv3 summary of DIR (no GPU)")
    ap.add_argument("--summarize-batched", default=None, metavar="DIR",
                    help="print the batched-path rocprofv3 summary of DIR (no GPU)")
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="no GPU: per-variant summary of the rocprofv3 runs in DIR, then exit")
    args = ap.parse_args()

    if args.summarize_profile:
        from paper_1708_01159_amd import profile_summary

        print(profile_summary.summarize(args.summarize_profile, ROOT))
        return
    if args.summarize_batched:
        from paper_1708_01159_amd import profile_summary

        print(profile_summary.summarize_batched(args.summarize_batched))
        return
    if args.summarize_components:
        from paper_1708_01159_amd import profile_summary

        print(profile_summary.summarize_components(args.summarize_components))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(asked for --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_01159_amd import graphgen as gg
    from paper_1708_01159_amd import gsw, trees

    if not os.path.exists(gsw.LIB_PATH) or not os.path.exists(gg._LIB):
        import __graft_entry__

        __graft_entry__.build()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    if args.components_only:
        line = {"components_pull": components_pull_only()}
        if args.copy_calib:
            line["copy_calibration"] = copy_calibration()
        print(json.dumps(line), flush=True)
        return

    if args.batched_only:
        sizes = tuple(int(x) for x in args.batched_only.split(","))
        line = {"batched": bench_batched(sizes)}
        if args.copy_calib:
            line["copy_calibration"] = copy_calibration()
        print(json.dumps(line), flush=True)
        return

    late = lambda: time.perf_counter() - T0 > args.budget
    t = time.perf_counter()
    g = gg.workload(args.workload)
    k_src, seed = gg.WORKLOAD_SOURCES[args.workload]
    if args.sources:
        k_src = args.sources
    srcs = gg.pick_sources(g, k_src, seed)
    log("graph %s n=%d nnz=%d built in %.1f s; %d sources" % (g.name, g.n, g.nnz, time.perf_counter() - t, len(srcs)))
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    tree = gsw.Tree.load(args.tree) if args.tree else trees.load_default()
    tree_name = os.path.basename(args.tree or trees.default_path())
    calls = [] if args.dispatch_log else None
    h = run_headline(args, g, G, tree, srcs, calls)

    extra, skipped = {}, []
    if not args.no_compare:
        fixed = run_fixed(G, srcs, h["m_c"], h["out_lv"], h["out_pa"])
        best_fixed = max(fixed, key=fixed.get)
        log("fixed kernels done; best %s %.2f GTEPS" % (best_fixed, fixed[best_fixed]))
        bpl = run_best_per_level(G, srcs, h["m_c"], h["med"], h["traces"], h["out_lv"], h["out_pa"],
                                 args.profile_reps, args.steps)
        log("best-per-level %.2f GTEPS; switched/best-per-level time %.4f; tree picked the fastest at %.1f%% of levels"
            % (bpl["gteps"], bpl["switched_time_over_best_per_level"], 100 * bpl["tree_agreement"]["fastest_picked"]))
        extra = {
            "fixed": fixed,
            "best_fixed": {"kernel": best_fixed, "gteps": fixed[best_fixed]},
            "switched_over_best_fixed": round(h["value"] / fixed[best_fixed], 3),
            "best_per_level": {"gteps": bpl["gteps"], "sources": bpl["sources"], "kernels": bpl["kernels"],
                               "profile_reps": bpl["profile_reps"],
                               "per_source_ratio_median": bpl["per_source_ratio_median"]},
            "switched_time_over_best_per_level": bpl["switched_time_over_best_per_level"],
            "tree_agreement": bpl["tree_agreement"],
        }

    if args.copy_calib:
        extra["copy_calibration"] = copy_calibration()

    sweep_graphs = {}
    if not args.no_compare:
        if not args.no_batched:
            if late():
                skipped.append("batched")
            else:
                extra["batched"] = optional_section("batched", bench_batched)
        if not args.no_sweep:
            if late():
                skipped.append("sweep")
            else:
                r = optional_section("sweep", bench_sweep, tree)
                if "error" in r:
                    extra["sweep"] = r
                else:
                    extra["sweep"], sweep_graphs = r
        cl_graph = None
        if not args.no_components:
            if late():
                skipped.append("components")
            else:
                cl = sweep_graphs.get("chunglu23") or gg.workload("chunglu23")
                cl_graph = (cl, gsw.Graph.from_csr(cl.offs, cl.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED))
                extra["components"] = optional_section("components", bench_components, tree,
                                                       {"rmat22": (g, G), "chunglu23": cl_graph})
        if not args.no_serving:
            if late():
                skipped.append("serving")
            else:
                pre = {"rmat22": (g, G)}
                if cl_graph is None:
                    cl = sweep_graphs.get("chunglu23") or gg.workload("chunglu23")
                    cl_graph = (cl, gsw.Graph.from_csr(cl.offs, cl.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED))
                pre["chunglu23"] = cl_graph
                extra["serving"] = optional_section("serving", bench_serving, tree, pre)
        if cl_graph is not None:
            cl_graph[1].close()
    if skipped:
        extra["skipped_for_time"] = skipped

    cpu = cpu_baseline(g, srcs, h["m_c"], args.cpu_budget)
    log("cpu oracle %.3f GTEPS" % cpu["value"])

    line = {
        "metric": METRIC, "value": round(h["value"], 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(h["wall"] / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "n": g.n, "nnz": g.nnz, "sources": len(srcs), "source_seed": int(seed),
                   "tree": tree_name, "policy": "tree-switched per level"},
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "kernel_time_share": h["shares"],
        "kernel_ms_per_source": round(h["kernel_ms"], 4),
        "median_source_ms": round(float(np.median(h["med"]) * 1e3), 4),
        "gteps_median_source": round(float(np.median(h["gteps_src"])), 3),
        "bench_seconds": round(time.perf_counter() - T0, 1),
    }
    line.update(extra)
    if calls is not None:
        with open(args.dispatch_log, "w") as f:
            json.dump(calls, f)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
