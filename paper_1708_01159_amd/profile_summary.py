"""Per-variant summary of a rocprofv3-profiled benchmark run (no GPU needed).

Every expansion variant runs inside one kernel, k_level_auto (or, for runs
of small levels, k_level_solo), so the profiler's per-kernel rows cannot
tell them apart.  The benchmark's ``--dispatch-log`` records, for every BFS
call, each level's kernel id, frontier size, algorithmic bytes (both byte
models), trace flags and the index of the launch that completed it.  Each
call starts with one k_init dispatch followed by its level-kernel launches
in order, so the launch index labels every level-kernel dispatch with the
variant it ran, for the kernel trace and for the FETCH_SIZE / WRITE_SIZE
counter runs alike.

The summary gives, for the dominant variant, the mean algorithmic bytes and
the mean rocprofv3 duration over the same set of dispatches (every call of
the profiled command: warm-up, timed steps and the instrumented pass over
all sources), so its roofline fraction can be recomputed from the summary
alone.  Counter bytes are scaled by what the same counters read for a plain
1 GiB device copy in the same run.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os

import numpy as np

EDGE_FUSE = 512  # the library's one-launch limit for push_edge frontiers
N_BASE = 11
PUSH_EDGE = 6
PROFILE_CMD = ("python3 -u bench.py --steps 2 --warmup 1 --no-compare --no-batched --no-sweep --no-serving "
               "--copy-calib --cpu-budget 1 --dispatch-log {d}/dispatch_log.json")
HBM_PEAK_GBS = 8000.0


def _csv_rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name):
    name = name.replace("gsw::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0][:48]


SOLO_FLAG = 4  # trace flag of a level run by a single-workgroup launch
LEVEL_KERNELS = ("k_level_auto", "k_level_solo")


def _align(dispatches, calls, names):
    """Label each dispatch (in start order) with (variant, bytes, literal bytes).

    Each call starts with one k_init dispatch, followed by its level-kernel
    dispatches (k_level_auto, k_level_solo) in launch order; every level's
    trace row names the launch that completed it.  A launch that completed
    one full-grid level is labelled with that level's kernel (a push_edge
    level on more than 512 entries also took the launch before it, its
    prefix sum); a single-workgroup launch with the levels it ran; a launch
    that completed none (the search had ended, or a single-workgroup launch
    handed its level on) as such."""
    labels = [None for _ in dispatches]
    starts = [i for i, d in enumerate(dispatches) if _short(d[0]) == "k_init"]
    if len(starts) != len(calls):
        raise SystemExit("profile has %d k_init dispatches, the dispatch log %d calls" % (len(starts), len(calls)))
    for c, (i0, call) in enumerate(zip(starts, calls)):
        i1 = starts[c + 1] if c + 1 < len(starts) else len(dispatches)
        mine = [i for i in range(i0 + 1, i1) if _short(dispatches[i][0]) in LEVEL_KERNELS]
        by_launch = {}
        for k, nf, b, lit, launch, flags in call["levels"]:
            by_launch.setdefault(launch, []).append((k, nf, b, lit, flags))
        if by_launch and max(by_launch) >= len(mine):
            raise SystemExit("call %d: launch %d logged, %d dispatched" % (c, max(by_launch), len(mine)))
        for j, i in enumerate(mine):
            lv = by_launch.get(j)
            if not lv:
                if labels[i] is None:
                    labels[i] = ("(no level completed)", None, None)
            elif any(f & SOLO_FLAG for *_, f in lv):
                labels[i] = ("single-workgroup launch", None, None)
            else:
                k, nf, b, lit, _ = lv[0]
                if k % N_BASE == PUSH_EDGE and nf > EDGE_FUSE:
                    labels[i] = (names[k] + " (expand)", b, None)
                    if j > 0:
                        labels[mine[j - 1]] = (names[k] + " (prefix)", None, None)
                else:
                    labels[i] = (names[k], b, lit)
    return labels


def summarize(d, root):
    from . import gsw

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
        return label[0] if label else _short(name)

    stat = {}
    for (n, t), l in zip(disp, lab):
        st = stat.setdefault(key(n, l), {"t": [], "f": [], "w": [], "b": [], "lit": []})
        st["t"].append(t)
        if l and l[1] is not None:
            st["b"].append(l[1])
        if l and l[2] is not None:
            st["lit"].append(l[2])
    for (n, v), l in zip(fe, fe_lab):
        stat.setdefault(key(n, l), {"t": [], "f": [], "w": [], "b": [], "lit": []})["f"].append(v)
    for (n, v), l in zip(wr, wr_lab):
        stat.setdefault(key(n, l), {"t": [], "f": [], "w": [], "b": [], "lit": []})["w"].append(v)
    rl = bench_line["roofline"]
    dom = rl["kernel"]
    sha = hashlib.sha256(open(os.path.join(root, "paper_1708_01159_amd", "csrc", "gsw_kernels.hip"), "rb")
                         .read()).hexdigest()
    L = ["# %s on R-MAT scale 22 (%d sources, tree-switched path)" % (dom, rl["sources"]), "",
         "Commands (from the repository root, `TMPDIR=/tmp`; the trace run's stdout is `trace_bench.json`):", "",
         "```",
         "rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace -o run -- ".format(d=d)
         + PROFILE_CMD.format(d=d),
         "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fetch -o run -- ".format(d=d) + PROFILE_CMD.format(d=d),
         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/write -o run -- ".format(d=d) + PROFILE_CMD.format(d=d),
         "python3 bench.py --summarize-profile " + d, "```", "",
         "Every dispatch of the command (warm-up, 2 timed steps, the event-timed pass), under the profiler. "
         "The level kernel's dispatches are attributed to the variant each ran from the dispatch log:", "",
         "| kernel / variant | dispatches | avg us | total us | FETCH_SIZE avg KB | WRITE_SIZE avg KB | algorithmic MB avg |",
         "|---|---:|---:|---:|---:|---:|---:|"]
    for k in sorted(stat, key=lambda k: -sum(stat[k]["t"])):
        st = stat[k]
        L.append("| %s | %d | %.2f | %.1f | %.1f | %.1f | %s |" % (
            k, len(st["t"]), np.mean(st["t"]) if st["t"] else 0, np.sum(st["t"]),
            np.mean(st["f"]) if st["f"] else 0, np.mean(st["w"]) if st["w"] else 0,
            "%.2f" % (np.mean(st["b"]) / 1e6) if st["b"] else "-"))
    s = stat[dom]
    fetched = np.mean(s["f"]) * 1024 * f_scale
    written = np.mean(s["w"]) * 1024 * w_scale
    traffic = fetched + written
    alg = float(np.mean(s["b"]))
    dur = float(np.mean(s["t"]))
    achieved = alg / (dur * 1e-6) / 1e9
    L += ["", "Counter scale from the plain 1 GiB device copy (`__amd_rocclr_copyBuffer`, 1 GiB read + "
          "1 GiB written): FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (f_scale, w_scale), "",
          "%s per launch, over the same %d dispatches:" % (dom, len(s["t"])), "",
          "* algorithmic bytes (library byte model): **%.2f MB**%s" % (
              alg / 1e6, "; the scope table's literal pull formula: %.2f MB" % (np.mean(s["lit"]) / 1e6)
              if s["lit"] else ""),
          "* rocprofv3 mean duration: **%.2f us** -> %.0f GB/s = **%.3f** of %.0f GB/s%s" % (
              dur, achieved, achieved / HBM_PEAK_GBS, HBM_PEAK_GBS,
              " (literal formula: %.3f)" % (np.mean(s["lit"]) / (dur * 1e-6) / 1e9 / HBM_PEAK_GBS)
              if s["lit"] else ""),
          "* HBM traffic (scaled counters): %.1f MB fetched + %.1f MB written = **%.1f MB**; "
          "traffic / algorithmic = %.2f" % (fetched / 1e6, written / 1e6, traffic / 1e6, traffic / alg),
          "* the bench line of this run (event-timed pass, its own launches): %.2f MB per launch, %.2f us, "
          "frac %.3f; value %.1f GTEPS (under the profiler)" % (
              rl["bytes_per_launch"] / 1e6, rl["mean_launch_ms"] * 1e3, rl["frac"], bench_line["value"]), "",
          "Machine-readable (read by bench.py while the kernel source is unchanged):", "", "```",
          "kernel: %s" % dom, "dispatches: %d" % len(s["t"]),
          "algorithmic_bytes_per_launch: %d" % alg, "mean_duration_us: %.3f" % dur,
          "frac_of_8tbs: %.4f" % (achieved / HBM_PEAK_GBS),
          "traffic_bytes_per_launch: %d" % traffic, "kernel_source_sha256: %s" % sha, "```"]
    return "\n".join(L)


BATCHED_CMD = "python3 -u bench.py --batched-only 1024 --copy-calib"
MS_KERNELS = ("k_ms_init", "k_ms_sources", "k_ms_push", "k_ms_level", "k_ms_finalize", "k_ms_transpose")


def summarize_batched(d, tuned_batches: int = 6):
    """Per-kernel summary of the batched path (R-MAT scale 20, 1024 sources)
    over the last ``tuned_batches`` batches of the profiled command (the
    tuned batch, run once untimed and five times timed; the autotuning
    batches before them are left out): rocprofv3 durations, FETCH_SIZE and
    WRITE_SIZE scaled by the 1 GiB copy of the same run, the traffic rate
    against 8 TB/s, and for the transpose -- a pure stream of B*n bytes in
    and B*n bytes out -- its algorithmic bytes and roofline fraction.  The
    level kernels' algorithmic bytes depend on each source's direction and
    on early exits that only the device sees, so their line gives the
    measured traffic."""
    line = json.loads(open(os.path.join(d, "trace_bench.json")).read().strip().splitlines()[-1])
    tr = sorted(_csv_rows(os.path.join(d, "trace", "run_kernel_trace.csv")), key=lambda r: int(r["Start_Timestamp"]))
    disp = [(_short(r["Kernel_Name"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3) for r in tr]

    def counters(sub, name):
        rows = [r for r in _csv_rows(os.path.join(d, sub, "run_counter_collection.csv")) if r["Counter_Name"] == name]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return [(_short(r["Kernel_Name"]), float(r["Counter_Value"])) for r in rows]

    fe, wr = counters("fetch", "FETCH_SIZE"), counters("write", "WRITE_SIZE")
    GiB = 1 << 30
    f_scale = GiB / (np.mean(sorted(v for n, v in fe if "copyBuffer" in n)[-2:]) * 1024)
    w_scale = GiB / (np.mean(sorted(v for n, v in wr if "copyBuffer" in n)[-2:]) * 1024)

    def last_batches(rows):
        starts = [i for i, r in enumerate(rows) if r[0] == "k_ms_init"]
        if len(starts) < tuned_batches:
            raise SystemExit("profile has %d batches, fewer than %d" % (len(starts), tuned_batches))
        i0 = starts[-tuned_batches]
        return [r for r in rows[i0:] if r[0] in MS_KERNELS]

    t_rows, f_rows, w_rows = last_batches(disp), last_batches(fe), last_batches(wr)
    B, n = 1024, 1 << 20
    info = line["batched"]["batches"][str(B)]
    L = ["# Batched multi-source BFS on R-MAT scale 20, %d sources" % B, "",
         "Commands (from the repository root, `TMPDIR=/tmp`; the trace run's stdout is `trace_bench.json`):", "",
         "```",
         "rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace -o run -- ".format(d=d) + BATCHED_CMD,
         "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fetch -o run -- ".format(d=d) + BATCHED_CMD,
         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/write -o run -- ".format(d=d) + BATCHED_CMD,
         "python3 bench.py --summarize-batched " + d, "```", "",
         "The tuned batch (thresholds %g / %g, block %d) runs once untimed and five times timed after the "
         "autotuning batches; the table covers those last %d batches, per batch.  The bench line of the trace "
         "run: %.3f ms per batch, %.1f GTEPS.  Counter scale from the plain 1 GiB device copy of the same run: "
         "FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (info["push_to_pull"], info["pull_to_push"], info["block_size"],
                                                    tuned_batches, info["ms"], info["gteps"], f_scale, w_scale), "",
         "| kernel | launches per batch | us per batch | fetched MB | written MB | traffic GB/s | of 8 TB/s |",
         "|---|---:|---:|---:|---:|---:|---:|"]
    per = {}
    for k in MS_KERNELS:
        t = [x for nm, x in t_rows if nm == k]
        f = [x for nm, x in f_rows if nm == k]
        w = [x for nm, x in w_rows if nm == k]
        if not t:
            continue
        us = sum(t) / tuned_batches
        fb = sum(f) * 1024 * f_scale / tuned_batches
        wb = sum(w) * 1024 * w_scale / tuned_batches
        rate = (fb + wb) / (us * 1e-6) / 1e9
        per[k] = (us, fb, wb)
        L.append("| %s | %.1f | %.1f | %.1f | %.1f | %.0f | %.3f |" % (
            k, len(t) / tuned_batches, us, fb / 1e6, wb / 1e6, rate, rate / HBM_PEAK_GBS))
    if "k_ms_transpose" in per:
        us, fb, wb = per["k_ms_transpose"]
        alg = 2.0 * B * n
        L += ["", "k_ms_transpose: algorithmic bytes %.1f MB per batch (the int8 levels, %d x %d bytes, read "
              "vertex-major and written source-major); %.1f us -> %.0f GB/s = **%.3f** of 8 TB/s; counter "
              "traffic / algorithmic = %.2f." % (alg / 1e6, B, n, us, alg / (us * 1e-6) / 1e9,
                                                 alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, (fb + wb) / alg)]
    return "\n".join(L)


COMPONENTS_CMD = "python3 -u bench.py --components-only --copy-calib"


def summarize_components(d):
    """The pull kernel of connected components (k_cc_pull) over the profiled
    command's calls: rocprofv3 mean duration, FETCH_SIZE and WRITE_SIZE per
    launch scaled by the 1 GiB copy of the same run, and the algorithmic
    bytes per launch from the command's own line (every launch reads every
    arc: 24 bytes per vertex with arcs plus 8 per arc)."""
    line = json.loads(open(os.path.join(d, "trace_bench.json")).read().strip().splitlines()[-1])
    info = line["components_pull"]
    tr = [r for r in _csv_rows(os.path.join(d, "trace", "run_kernel_trace.csv"))]
    durs = {}
    for r in tr:
        durs.setdefault(_short(r["Kernel_Name"]), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)

    def counters(sub, name):
        out = {}
        for r in _csv_rows(os.path.join(d, sub, "run_counter_collection.csv")):
            if r["Counter_Name"] == name:
                out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return out

    fe, wr = counters("fetch", "FETCH_SIZE"), counters("write", "WRITE_SIZE")
    GiB = 1 << 30
    cb = [k for k in fe if "copyBuffer" in k][0]
    f_scale = GiB / (np.mean(sorted(fe[cb])[-2:]) * 1024)
    w_scale = GiB / (np.mean(sorted(wr[cb])[-2:]) * 1024)
    L = ["# Connected components on R-MAT scale 22: the pull propagation kernel", "",
         "Commands (from the repository root, `TMPDIR=/tmp`; the trace run's stdout is `trace_bench.json`):", "",
         "```",
         "rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace -o run -- ".format(d=d) + COMPONENTS_CMD,
         "rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fetch -o run -- ".format(d=d) + COMPONENTS_CMD,
         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/write -o run -- ".format(d=d) + COMPONENTS_CMD,
         "python3 bench.py --summarize-components " + d, "```", "",
         "%d calls of gsw_cc with propagation alone and the pull kernel at every iteration (%d iterations per "
         "call; labels equal to the oracle: %s).  Every launch of k_cc_pull reads the rows of all %d vertices "
         "with arcs and all %d arcs.  Counter scale from the plain 1 GiB device copy of the same run: "
         "FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (info["calls"], info["iterations_per_call"],
                                                    info["equal_to_oracle"], info["n_rest"], info["e_rest"],
                                                    f_scale, w_scale), "",
         "| kernel | dispatches | avg us | FETCH_SIZE avg KB | WRITE_SIZE avg KB |", "|---|---:|---:|---:|---:|"]
    for k in sorted(durs, key=lambda k: -sum(durs[k])):
        if not k.startswith("k_cc"):
            continue
        L.append("| %s | %d | %.2f | %.1f | %.1f |" % (k, len(durs[k]), np.mean(durs[k]),
                                                      np.mean(fe.get(k, [0.0])), np.mean(wr.get(k, [0.0]))))
    us = float(np.mean(durs["k_cc_pull"]))
    alg = info["bytes_per_iteration"]
    traffic = (np.mean(fe["k_cc_pull"]) * f_scale + np.mean(wr["k_cc_pull"]) * w_scale) * 1024
    L += ["", "k_cc_pull per launch: algorithmic %.1f MB; rocprofv3 mean %.1f us -> %.0f GB/s = **%.3f** of "
          "8 TB/s; HBM traffic (scaled counters) %.1f MB, traffic / algorithmic = %.2f; the events of the bench "
          "line: %.1f us per iteration." % (alg / 1e6, us, alg / (us * 1e-6) / 1e9,
                                             alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, traffic / 1e6, traffic / alg,
                                             info["mean_iteration_ms_events"] * 1e3)]
    return "\n".join(L)
