#!/usr/bin/env python3
"""Benchmark: GTEPS of tree-switched BFS on R-MAT scale 22 vs every fixed
kernel and the best-per-level schedule, on one MI355X.

One step = a tree-switched BFS (level loop, per-level kernel choice, every
expansion kernel it picks) from each of the 64 seeded sources of the
workload.  GTEPS of a source = undirected edges of its component / time of
its gsw_bfs call (graph upload and result copy-back excluded, as in the
paper's measurements); the reported value is the harmonic mean over sources
of each source's median over the timed steps.

Prints ONE JSON line.  Besides the contract fields:
  fixed            harmonic-mean GTEPS of each kernel used at every level
  best_per_level   GTEPS of replaying, per source, the fastest kernel of each
                   level (times measured from the same saved BFS state)
  tree_agreement   share of levels where the tree picked that fastest kernel
  roofline         the dominant kernel of the switched path: algorithmic bytes
                   per launch / mean launch time, the time taken from the
                   library's per-level device timers (the level's first
                   workgroup stamps the GPU's constant-rate wall clock when it
                   starts, the level's last workgroup reads it when it ends)
                   in one instrumented pass over the same sources right after
                   the timed steps; traffic = HBM bytes per launch from the
                   committed rocprofv3 counter summary, while the kernel
                   source it was taken on is unchanged
  cpu_baseline     the CPU oracle on a bounded sample of the same sources

Profiling: every expansion variant runs inside one kernel (k_level_auto),
so rocprofv3's per-kernel view cannot tell them apart.  ``--dispatch-log``
records, for every BFS call, the kernel and frontier size of each level;
``--summarize-profile DIR`` (no GPU) aligns the per-dispatch rows of the
kernel trace and of the FETCH_SIZE / WRITE_SIZE counter runs in DIR with
that log -- each call starts with one k_init dispatch, then each level takes
one k_level_auto launch (two for push_edge on more than 512 entries), the
rest of the call's launches find the search ended -- and prints the
per-variant summary kept under profiles/.  ``--batched-only 1024`` runs only
the batched section (for a kernel-trace profile of the batched kernels).
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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
    return {"value": round(hmean(gteps), 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": "%d of %d sources of the same workload, single-threaded FIFO BFS, %.1f s"
                      % (len(times), len(srcs), sum(times)),
            "cpu": cpu_model()}


def counter_traffic(kernel_name):
    """HBM bytes per launch of ``kernel_name`` from the committed rocprofv3
    counter summary, or None when that summary is missing, is for another
    kernel, or was taken on a different kernel source."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_rmat22.md" % kernel_name)
    src = os.path.join(ROOT, "paper_1708_01159_amd", "csrc", "gsw_kernels.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and
                  line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel", "kernel_source_sha256"))
    if fields.get("kernel") != kernel_name or fields.get("kernel_source_sha256") != sha:
        return None
    return int(fields["traffic_bytes_per_launch"])


def timed(runner, src, sync):
    sync()
    t0 = time.perf_counter()
    runner.run(int(src))
    return time.perf_counter() - t0


def bench_batched(log, batches=(64, 256, 1024)):
    """Batched multi-source BFS on R-MAT scale 20 vs the same sources one at a
    time on the tree-switched single-source path."""
    import torch

    from paper_1708_01159_amd import autotune, gsw, serve, trees
    from paper_1708_01159_amd import graphgen as gg

    sync = torch.cuda.synchronize
    g = gg.workload("rmat20")
    k, seed = gg.WORKLOAD_SOURCES["rmat20"]
    srcs = gg.pick_sources(g, max(batches), seed)
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
        p2p, p2s, table = autotune.tune(G, src, log=None)
        lvB = torch.empty((B, g.n), dtype=torch.int8, device="cuda")
        gsw.msbfs(G, src, p2p, p2s, out=lvB)
        ts = []
        for _ in range(3):
            sync()
            t0 = time.perf_counter()
            _, nl = gsw.msbfs(G, src, p2p, p2s, out=lvB)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        edges = int(ce[src].sum())
        one = float(t_single[:B].sum())
        out[str(B)] = {"ms": round(t * 1e3, 3), "gteps": round(edges / t / 1e9, 2),
                       "push_to_pull": p2p, "pull_to_push": p2s,
                       "one_at_a_time_ms": round(one * 1e3, 3),
                       "one_at_a_time_gteps": round(edges / one / 1e9, 2),
                       "speedup": round(one / t, 2), "levels": nl}
        log("batched B=%d: %.2f ms (%.1f GTEPS) vs one at a time %.2f ms (%.1f GTEPS); thresholds %g/%g"
            % (B, t * 1e3, edges / t / 1e9, one * 1e3, edges / one / 1e9, p2p, p2s))
    G.close()
    return {"workload": "R-MAT scale 20 (1,048,576 vertices), edgefactor 16, seed 6; sources seed 106",
            "level_type": "int8", "thresholds": "autotuned per batch size", "batches": out}


def bench_sweep(tree, args, log):
    """Structure sweep: switched vs every fixed kernel vs best-per-level."""
    import torch

    from paper_1708_01159_amd import gsw
    from paper_1708_01159_amd import graphgen as gg

    sync = torch.cuda.synchronize
    res = {}
    for name, prof_src in (("grid2048_del5", 2), ("chunglu23", 8), ("er22", 8)):
        t = time.perf_counter()
        g = gg.workload(name)
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
        fixed = {}
        for kern in range(gsw.N_KERNELS):
            fx = gsw.Runner(G, lv, None, policy="fixed", kernel=kern, trace_cap=1 << 16)
            ts = np.array([timed(fx, s, sync) for s in srcs])
            fixed[gsw.KERNEL_NAMES[kern]] = round(hmean(m_c / ts / 1e9), 3)
        bf = max(fixed, key=fixed.get)
        sched = gsw.Runner(G, lv, None, policy="schedule", schedule=[0], trace_cap=1 << 16)
        r_sw, r_bpl = [], []
        for i, s in enumerate(srcs[:prof_src]):
            times, _, _ = gsw.bfs_profile(G, int(s), reps=2, advance_kernel=-1)
            sched.set_schedule(np.argmin(times, axis=1).astype(np.int32))
            sched.run(int(s))
            r_bpl.append(min(timed(sched, s, sync), timed(sched, s, sync)))
            r_sw.append(t_sw[i])
        gt = hmean(m_c / t_sw / 1e9)
        res[name] = {"n": g.n, "nnz": g.nnz, "sources": len(srcs), "switched_gteps": round(gt, 3),
                     "fixed": fixed, "best_fixed": bf, "switched_over_best_fixed": round(gt / fixed[bf], 3),
                     "switched_time_over_best_per_level": round(float(np.sum(r_sw) / np.sum(r_bpl)), 4),
                     "best_per_level_sources": prof_src}
        log("sweep %s: switched %.2f GTEPS, best fixed %s %.2f, vs best-per-level %.3f (%.0f s)"
            % (name, gt, bf, fixed[bf], res[name]["switched_time_over_best_per_level"],
               time.perf_counter() - t))
        G.close()
    return res


def bench_serving(args, tree, log, preloaded):
    """Continuous-batching serving vs one query at a time, p50/p99 latency."""
    from paper_1708_01159_amd import gsw, serve
    from paper_1708_01159_amd import graphgen as gg

    if args.serving_full:
        specs = [("rmat16", lambda: gg.rmat(16, 16, seed=7)), ("rmat18", lambda: gg.rmat(18, 16, seed=8)),
                 ("rmat20", lambda: gg.rmat(20, 16, seed=9)), ("rmat22", lambda: gg.rmat(22, 16, seed=10)),
                 ("rmat24", lambda: gg.rmat(24, 16, seed=11)), ("grid4096", lambda: gg.grid(4096, 4096, 0.0, seed=12)),
                 ("chunglu23", lambda: gg.chung_lu(1 << 23, 2.1, 20.0, seed=13)),
                 ("er24", lambda: gg.erdos_renyi(1 << 24, 4 << 24, seed=14))]
        rates, duration, slots = (100, 500, 1000, 2000, 5000, 12000), 5.0, 64
        budget = 48 << 30
    else:
        specs = [("rmat22", None), ("rmat20", lambda: gg.rmat(20, 16, seed=9)),
                 ("er20", lambda: gg.erdos_renyi(1 << 20, 4 << 20, seed=14))]
        rates, duration, slots = (500, 2000, 6000), 2.0, 64
        budget = 16 << 30
    residents, cands = {}, {}
    for name, make in specs:
        if make is None:
            g, G = preloaded[name]
        else:
            g = make()
            G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
        residents[name] = serve.Resident(name, G, serve.component_edges(g.offs, g.cols))
        cands[name] = np.flatnonzero(g.degrees() > 0)
    names = [s[0] for s in specs]
    runs = []
    fmt = lambda r: "p50 %.2f p99 %.2f ms %.1f GTEPS" % (r["p50_ms"], r["p99_ms"], r["gteps"])
    for rate in rates:
        trace = serve.poisson_trace(rate, duration, names, cands, seed=107 + rate)
        row = {"rate_qps": rate}
        for key, solo in (("batched", False), ("batched_solo_lane", True)):
            srv = serve.Server(residents, slots=slots, hbm_budget=budget, solo=solo, solo_factory=None)
            qb = srv.run(trace, timeout_s=120)
            row[key] = serve.summarize(qb, residents, "continuous batching" +
                                       (" + single-source lane" if solo else ""))
            if solo:
                row[key]["solo_served"] = srv.solo_served
            log("serving %d QPS, %s done" % (rate, key))  # one line per mode: a long drain still reports
        if not args.serving_full or rate <= 500:
            qo = serve.serve_one_at_a_time(residents, trace, tree, timeout_s=120)
            row["one_at_a_time"] = serve.summarize(qo, residents, "one at a time")
        runs.append(row)
        log("serving %d QPS: batched %s; + solo lane %s; one at a time %s"
            % (rate, fmt(row["batched"]), fmt(row["batched_solo_lane"]),
               fmt(row["one_at_a_time"]) if "one_at_a_time" in row else "-"))
    return {"graphs": names, "zipf": 1.1, "duration_s": duration, "slots": slots,
            "hbm_budget_bytes": budget, "runs": runs}


EDGE_FUSE = 512  # the library's one-launch limit for push_edge frontiers
PROFILE_CMD = ("python3 -u bench.py --steps 2 --warmup 1 --no-compare --copy-calib --cpu-budget 1 "
               "--dispatch-log {d}/dispatch_log.json")


def _csv_rows(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name):
    name = name.replace("gsw::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0][:48]


def _align(dispatches, calls, names):
    """Label each dispatch (in start order) with the variant it ran."""
    labels = ["" for _ in dispatches]
    starts = [i for i, d in enumerate(dispatches) if _short(d[0]) == "k_init"]
    if len(starts) != len(calls):
        raise SystemExit("profile has %d k_init dispatches, the dispatch log %d calls" % (len(starts), len(calls)))
    for c, (i0, call) in enumerate(zip(starts, calls)):
        i1 = starts[c + 1] if c + 1 < len(starts) else len(dispatches)
        mine = [i for i in range(i0 + 1, i1) if _short(dispatches[i][0]) == "k_level_auto"]
        want = []
        for k, nf in call["levels"]:
            if k == 6 and nf > EDGE_FUSE:
                want += ["push_edge (prefix)", "push_edge (expand)"]
            else:
                want.append(names[k])
        if len(want) > len(mine):
            raise SystemExit("call %d: %d level launches logged, %d dispatched" % (c, len(want), len(mine)))
        for j, i in enumerate(mine):
            labels[i] = want[j] if j < len(want) else "(search ended)"
    return labels


def summarize_profile(d):
    """Per-variant summary of a profiled run (see the module docstring)."""
    import hashlib

    from paper_1708_01159_amd import gsw

    calls = json.load(open(os.path.join(d, "dispatch_log.json")))
    bench_line = json.loads(open(os.path.join(d, "trace_bench.json")).read().strip().splitlines()[-1])
    tr = sorted(_csv_rows(os.path.join(d, "trace", "run_kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    disp = [(r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3) for r in tr]
    lab = _align(disp, calls, gsw.KERNEL_NAMES)

    def counters(sub, name):
        rows = [r for r in _csv_rows(os.path.join(d, sub, "run_counter_collection.csv")) if r["Counter_Name"] == name]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        vals = [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]
        return vals, _align(vals, calls, gsw.KERNEL_NAMES)

    fe, fe_lab = counters("fetch", "FETCH_SIZE")
    wr, wr_lab = counters("write", "WRITE_SIZE")
    GiB = 1 << 30
    copy_f = sorted(v for n, v in fe if "copyBuffer" in n)[-2:]
    copy_w = sorted(v for n, v in wr if "copyBuffer" in n)[-2:]
    f_scale = GiB / (np.mean(copy_f) * 1024)
    w_scale = GiB / (np.mean(copy_w) * 1024)

    def key(name, label):
        return label if label else _short(name)

    stat = {}
    for (n, t), l in zip(disp, lab):
        stat.setdefault(key(n, l), {"t": [], "f": [], "w": []})["t"].append(t)
    for (n, v), l in zip(fe, fe_lab):
        stat.setdefault(key(n, l), {"t": [], "f": [], "w": []})["f"].append(v)
    for (n, v), l in zip(wr, wr_lab):
        stat.setdefault(key(n, l), {"t": [], "f": [], "w": []})["w"].append(v)
    L = ["# pull_bitmap on R-MAT scale 22 (64 sources, tree-switched path)", "",
         "Commands (from the repository root, `TMPDIR=/tmp`; the trace run's stdout is `trace_bench.json`):", "",
         "```",
         "rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace -o run -- ".format(d=d)
         + PROFILE_CMD.format(d=d),
         "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fetch -o run -- ".format(d=d) + PROFILE_CMD.format(d=d),
         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/write -o run -- ".format(d=d) + PROFILE_CMD.format(d=d),
         "python3 bench.py --summarize-profile " + d, "```", "",
         "Every dispatch of the command (warm-up, 2 timed steps, the instrumented pass), under the profiler. "
         "The level kernel's dispatches are attributed to the variant each ran from the dispatch log:", "",
         "| kernel / variant | dispatches | avg us | total us | FETCH_SIZE avg KB | WRITE_SIZE avg KB |",
         "|---|---:|---:|---:|---:|---:|"]
    for k in sorted(stat, key=lambda k: -sum(stat[k]["t"])):
        st = stat[k]
        L.append("| %s | %d | %.2f | %.1f | %.1f | %.1f |" % (
            k, len(st["t"]), np.mean(st["t"]) if st["t"] else 0, np.sum(st["t"]),
            np.mean(st["f"]) if st["f"] else 0, np.mean(st["w"]) if st["w"] else 0))
    pull = stat["pull_bitmap"]
    traffic = np.mean(pull["f"]) * 1024 * f_scale + np.mean(pull["w"]) * 1024 * w_scale
    rl = bench_line["roofline"]
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1708_01159_amd", "csrc", "gsw_kernels.hip"), "rb")
                         .read()).hexdigest()
    L += ["", "Counter scale from the plain 1 GiB device copy (`__amd_rocclr_copyBuffer`, 1 GiB read + "
          "1 GiB written): FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (f_scale, w_scale), "",
          "pull_bitmap per launch:", "",
          "* HBM traffic (scaled counters): %.1f MB fetched + %.1f MB written = **%.1f MB**" % (
              np.mean(pull["f"]) * 1024 * f_scale / 1e6, np.mean(pull["w"]) * 1024 * w_scale / 1e6, traffic / 1e6),
          "* algorithmic bytes (bench byte model, sampled launches): %.1f MB; traffic / algorithmic = %.2f" % (
              rl["bytes_per_launch"] / 1e6, traffic / rl["bytes_per_launch"]),
          "* mean duration: rocprofv3 %.2f us over %d dispatches; bench (device wall-clock stamps, same run) "
          "%.2f us over %d launches" % (np.mean(pull["t"]), len(pull["t"]), rl["mean_launch_ms_all"] * 1e3,
                                        rl["launches_all"]),
          "* bench line of this run: value %.1f GTEPS (under the profiler), roofline achieved %.0f GB/s "
          "(frac %.3f)" % (bench_line["value"], rl["achieved"], rl["frac"]), "",
          "Machine-readable (read by bench.py while the kernel source is unchanged):", "", "```",
          "traffic_bytes_per_launch: %d" % traffic, "kernel: pull_bitmap", "kernel_source_sha256: %s" % sha, "```"]
    print("\n".join(L))


def _logged(runner, tag, calls):
    """Runner whose every call appends its levels' (kernel, frontier) to calls."""
    if calls is None:
        return runner
    run = runner.run

    def logged_run(source):
        n = run(source)
        calls.append({"tag": tag, "source": int(source),
                      "levels": [[r.kernel, r.n_frontier] for r in runner.rows()]})
        return n

    runner.run = logged_run
    return runner


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=None, help="override the source count")
    ap.add_argument("--tree", default=None, help="tree JSON (default: shipped tree)")
    ap.add_argument("--no-compare", action="store_true",
                    help="only the timed switched path (used for profiling runs)")
    ap.add_argument("--profile-reps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--roofline-sources", type=int, default=4)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-source section")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serving-full", action="store_true",
                    help="serving over the 8-graph set (RMAT 16-24, 4096^2 grid, Chung-Lu 2^23, "
                         "ER 2^24) at 100-5000 QPS instead of the short default")
    ap.add_argument("--sweep", action="store_true",
                    help="also the structure sweep: grid 2048^2 (5%% deleted), Chung-Lu 2^23, ER 2^22")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    ap.add_argument("--dispatch-log", default=None,
                    help="write every BFS call's (kernel, frontier) per level to this JSON file")
    ap.add_argument("--batched-only", default=None, metavar="B[,B...]",
                    help="only the batched section at these batch sizes (one JSON line; for profiling)")
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="no GPU: per-variant summary of the rocprofv3 runs in DIR, then exit")
    args = ap.parse_args()

    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(asked for --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_01159_amd import graphgen as gg
    from paper_1708_01159_amd import gsw, traffic, trees

    if not os.path.exists(gsw.LIB_PATH) or not os.path.exists(gg._LIB):
        import __graft_entry__

        __graft_entry__.build()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize

    if args.batched_only:
        sizes = tuple(int(x) for x in args.batched_only.split(","))
        print(json.dumps({"batched": bench_batched(log, sizes)}), flush=True)
        return

    t = time.perf_counter()
    g = gg.workload(args.workload)
    k_src, seed = gg.WORKLOAD_SOURCES[args.workload]
    if args.sources:
        k_src = args.sources
    srcs = gg.pick_sources(g, k_src, seed)
    log("graph %s n=%d nnz=%d built in %.1f s; %d sources" % (g.name, g.n, g.nnz,
                                                              time.perf_counter() - t, len(srcs)))
    G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
    tree = gsw.Tree.load(args.tree) if args.tree else trees.load_default()
    tree_name = os.path.basename(args.tree or trees.default_path())
    n = g.n
    out_lv = torch.empty((1, n), dtype=torch.int32, device="cuda")
    out_pa = torch.empty((1, n), dtype=torch.int32, device="cuda")
    deg = g.degrees()
    calls = [] if args.dispatch_log else None
    sw = _logged(gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree), "switched", calls)
    # the same path with the per-level device timers on (kept out of the
    # timed steps)
    sw_ev = _logged(gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree, time_levels=True), "timed levels",
                    calls)

    # warm-up (also: component sizes from the GPU's own levels, and the level
    # arrays of the first few sources for the byte model)
    m_c = np.zeros(len(srcs), dtype=np.int64)
    keep_lv = {}
    for w in range(max(args.warmup, 1)):
        for i, s in enumerate(srcs):
            sw.run(int(s))
            if w == 0:
                lv = out_lv[0].cpu().numpy()
                m_c[i] = int(deg[lv >= 0].sum() // 2)
                if i < args.roofline_sources:
                    keep_lv[i] = lv.copy()
    log("warm-up done")

    # timed region: K steps of the tree-switched path over every source
    per_src = np.zeros((args.steps, len(srcs)))
    traces = []
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
    ms_per_step = wall / args.steps * 1e3
    log("switched: %.2f GTEPS (harmonic), %.2f ms/step, %.3f ms median source"
        % (value, ms_per_step, np.median(med) * 1e3))
    # instrumented pass over the same sources: per-level kernel times
    per_src_ev = np.zeros(len(srcs))
    for i, s in enumerate(srcs):
        per_src_ev[i] = timed(sw_ev, s, sync)
        traces.append((i, sw_ev.rows()))

    # dominant kernel of the timed region and its roofline
    ktime = np.zeros(gsw.N_KERNELS)
    kcount = np.zeros(gsw.N_KERNELS, dtype=np.int64)
    for _, tr in traces:
        for r in tr:
            ktime[r.kernel] += r.ms
            kcount[r.kernel] += 1
    dom = int(np.argmax(ktime))
    b_sum, t_sum, launches = 0, 0.0, 0
    for i, tr in traces:
        if i not in keep_lv:
            continue
        lv = keep_lv[i]
        nf, ef = traffic.level_sizes(g.offs, lv)
        for r in tr:
            if r.kernel == dom:
                b_sum += traffic.level_bytes(dom, g.offs, g.cols, lv, r.level, nf, ef)
                t_sum += r.ms * 1e-3
                launches += 1
    achieved = b_sum / t_sum / 1e9 if t_sum > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": gsw.KERNEL_NAMES[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": counter_traffic(gsw.KERNEL_NAMES[dom]),
                "bytes_per_launch": int(b_sum / max(launches, 1)),
                "mean_launch_ms": round(t_sum / max(launches, 1) * 1e3, 4),
                "launches_sampled": launches,
                "mean_launch_ms_all": round(float(ktime[dom] / max(kcount[dom], 1)), 4),
                "launches_all": int(kcount[dom]),
                "share_of_kernel_time": round(float(ktime[dom] / ktime.sum()), 3)}
    kernel_ms = float(ktime.sum() / len(srcs))
    roofline["instrumented_pass_median_source_ms"] = round(float(np.median(per_src_ev)) * 1e3, 4)

    extra = {}
    if not args.no_compare:
        fixed = {}
        for kern in range(gsw.N_KERNELS):
            fx = gsw.Runner(G, out_lv, out_pa, policy="fixed", kernel=kern)
            fx.run(int(srcs[0]))  # warm
            ts = np.array([timed(fx, s, sync) for s in srcs])
            fixed[gsw.KERNEL_NAMES[kern]] = round(hmean(m_c / ts / 1e9), 3)
            log("fixed %-12s %.2f GTEPS" % (gsw.KERNEL_NAMES[kern], fixed[gsw.KERNEL_NAMES[kern]]))
        best_fixed = max(fixed, key=fixed.get)
        # best-per-level schedule: fastest kernel per level from the same saved state
        t_bpl, agree, levels_total, regret = [], 0, 0, 0.0
        sched_runner = gsw.Runner(G, out_lv, out_pa, policy="schedule", schedule=[0])
        last_trace = dict(traces)  # the last timed step's choices per source
        for i, s in enumerate(srcs):
            times, _, _ = gsw.bfs_profile(G, int(s), reps=args.profile_reps, advance_kernel=-1)
            sched = np.argmin(times, axis=1).astype(np.int32)
            sched_runner.set_schedule(sched)
            sched_runner.run(int(s))
            t_bpl.append(np.median([timed(sched_runner, s, sync) for _ in range(max(args.steps, 1))]))
            picks = [r.kernel for r in last_trace[i]]
            for d, kk in enumerate(picks[:len(sched)]):
                agree += int(kk == sched[d])
                regret += float(times[d, kk] - times[d, sched[d]])
                levels_total += 1
        t_bpl = np.array(t_bpl)
        gteps_bpl = hmean(m_c / t_bpl / 1e9)
        extra = {
            "fixed": fixed,
            "best_fixed": {"kernel": best_fixed, "gteps": fixed[best_fixed]},
            "switched_over_best_fixed": round(value / fixed[best_fixed], 3),
            "best_per_level": {"gteps": round(gteps_bpl, 3)},
            "switched_time_over_best_per_level": round(float(med.sum() / t_bpl.sum()), 4),
            "tree_agreement": {"levels": levels_total, "fastest_picked": round(agree / max(levels_total, 1), 3),
                               "mean_regret_ms_per_source": round(regret / len(srcs), 4)},
        }
        log("best fixed %s %.2f; best-per-level %.2f GTEPS; tree picked the fastest at %d/%d levels"
            % (best_fixed, fixed[best_fixed], gteps_bpl, agree, levels_total))

    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b.copy_(a)
        ev0.record()
        b.copy_(a)
        ev1.record()
        sync()
        ms = ev0.elapsed_time(ev1)
        extra["copy_calibration"] = {"bytes_read": a.numel() * 4, "bytes_written": a.numel() * 4,
                                     "ms": round(ms, 4), "gbs": round(2 * a.numel() * 4 / ms / 1e6, 1)}
        del a, b

    if not args.no_batched and not args.no_compare:
        extra["batched"] = bench_batched(log)
    if args.sweep:
        extra["sweep"] = bench_sweep(tree, args, log)
    if not args.no_serving and not args.no_compare:
        extra["serving"] = bench_serving(args, tree, log, {"rmat22": (g, G)})

    cpu = cpu_baseline(g, srcs, m_c, args.cpu_budget)
    log("cpu oracle %.3f GTEPS" % cpu["value"])

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT.get(args.workload, args.workload),
                   "n": g.n, "nnz": g.nnz, "sources": len(srcs), "source_seed": int(seed),
                   "tree": tree_name, "policy": "tree-switched per level"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_time_share": {gsw.KERNEL_NAMES[k]: round(float(ktime[k] / ktime.sum()), 3)
                              for k in range(gsw.N_KERNELS) if kcount[k]},
        "kernel_ms_per_source": round(kernel_ms, 4),
        "median_source_ms": round(float(np.median(med) * 1e3), 4),
        "gteps_median_source": round(float(np.median(gteps_src)), 3),
    }
    line.update(extra)
    if calls is not None:
        with open(args.dispatch_log, "w") as f:
            json.dump(calls, f)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
