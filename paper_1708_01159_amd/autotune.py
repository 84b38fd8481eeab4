"""Autotuner for the batched BFS: direction thresholds and block size.

The batched traversal switches a source from top-down to bottom-up when its
frontier's arcs exceed ``push_to_pull`` of the arcs it has not reached yet,
and back when they drop below ``pull_to_push`` of all arcs; its level
kernels run in workgroups of ``block_size`` threads.  The best settings
depend on the graph and the batch size, so they are measured: every
threshold pair runs the same sample batch at the default block size, then
every block size runs with the fastest pair, and the fastest is kept.  The
sample should be a batch of sources other than the ones to be timed.
Results are cached per (graph signature, batch size) in a JSON file when a
path is given.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import gsw

PUSH_TO_PULL = (0.001, 0.003, 0.01, 0.03, 0.07, 0.2)
PULL_TO_PUSH = (0.0001, 0.001, 0.01)
BLOCK_SIZES = (128, 256, 512)
DEFAULT_BLOCK = 256


def signature(graph: gsw.Graph, batch: int) -> str:
    info = graph.info()
    st = [round(x, 1) for x in info["deg_stats"]]
    return "n%d_m%d_deg%s_b%d" % (info["n"], info["nnz"], "-".join(map(str, st)), batch)


def _time(graph, sources, a, b, bs, out, reps):
    import torch

    gsw.msbfs(graph, sources, a, b, out=out, block_size=bs)  # warm (and capture)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gsw.msbfs(graph, sources, a, b, out=out, block_size=bs)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune(graph: gsw.Graph, sources, reps: int = 3, cache_path: str = None, log=None):
    """Returns (push_to_pull, pull_to_push, block_size, table) for batches
    like ``sources``; table rows are (push_to_pull, pull_to_push, block, s)."""
    import torch

    key = signature(graph, len(sources))
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            c = cache[key]
            return c["push_to_pull"], c["pull_to_push"], c["block_size"], c["table"]
    out = torch.empty((len(sources), graph.n), dtype=torch.int8, device="cuda")
    table = []
    for a in PUSH_TO_PULL:
        for b in PULL_TO_PUSH:
            if b >= a:
                continue
            table.append((a, b, DEFAULT_BLOCK, _time(graph, sources, a, b, DEFAULT_BLOCK, out, reps)))
            if log:
                log("autotune push_to_pull=%g pull_to_push=%g: %.3f ms" % (a, b, table[-1][3] * 1e3))
    a, b, _, _ = min(table, key=lambda r: r[3])
    for bs in BLOCK_SIZES:
        if bs != DEFAULT_BLOCK:
            table.append((a, b, bs, _time(graph, sources, a, b, bs, out, reps)))
            if log:
                log("autotune block_size=%d: %.3f ms" % (bs, table[-1][3] * 1e3))
    a, b, bs, _ = min(table, key=lambda r: r[3])
    if cache_path:
        cache[key] = dict(push_to_pull=a, pull_to_push=b, block_size=bs, table=table)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return a, b, bs, table
