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
                   library's per-level device timers (every workgroup of the
                   level's kernel stamps the GPU's constant-rate wall clock at
                   entry and exit; the level lasts from the first entry to the
                   last exit) in one instrumented pass over the same sources
                   right after the timed steps; traffic = HBM bytes per launch
                   from the committed rocprofv3 counter summary, while the
                   kernel source it was taken on is unchanged
  cpu_baseline     the CPU oracle on a bounded sample of the same sources
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22")
    ap.add_argument("--sources", type=int, default=None, help="override the source count")
    ap.add_argument("--tree", default=None, help="tree JSON (default: shipped tree)")
    ap.add_argument("--no-compare", action="store_true",
                    help="only the timed switched path (used for profiling runs)")
    ap.add_argument("--profile-reps", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--roofline-sources", type=int, default=4)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()

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
    sw = gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree)
    # the same path with HIP events around every level's kernels (about 6 us
    # of host time per level, so it is kept out of the timed steps)
    sw_ev = gsw.Runner(G, out_lv, out_pa, policy="tree", tree=tree, time_levels=True)

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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
