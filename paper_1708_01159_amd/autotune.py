"""Autotuner for the batched BFS's direction thresholds.

The batched traversal switches a source from top-down to bottom-up when its
frontier's arcs exceed ``push_to_pull`` of the arcs it has not reached yet,
and back when they drop below ``pull_to_push`` of all arcs.  The best pair depends on the graph and the batch size, so
it is measured: every candidate pair runs the same sample batch and the
fastest is kept.  Results are cached per (graph signature, batch size) in a
JSON file when a path is given.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import gsw

PUSH_TO_PULL = (0.001, 0.003, 0.01, 0.03, 0.07, 0.2)
PULL_TO_PUSH = (0.0001, 0.001, 0.01)


def signature(graph: gsw.Graph, batch: int) -> str:
    info = graph.info()
    st = [round(x, 1) for x in info["deg_stats"]]
    return "n%d_m%d_deg%s_b%d" % (info["n"], info["nnz"], "-".join(map(str, st)), batch)


def tune(graph: gsw.Graph, sources, reps: int = 2, cache_path: str = None, log=None):
    """Returns (push_to_pull, pull_to_push, table) for batches like ``sources``."""
    import torch

    key = signature(graph, len(sources))
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            c = cache[key]
            return c["push_to_pull"], c["pull_to_push"], c["table"]
    out = torch.empty((len(sources), graph.n), dtype=torch.int8, device="cuda")
    table = []
    for a in PUSH_TO_PULL:
        for b in PULL_TO_PUSH:
            if b >= a:
                continue
            gsw.msbfs(graph, sources, a, b, out=out)  # warm
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                gsw.msbfs(graph, sources, a, b, out=out)
                ts.append(time.perf_counter() - t0)
            table.append((a, b, float(np.median(ts))))
            if log:
                log("autotune push_to_pull=%g pull_to_push=%g: %.3f ms" % (a, b, table[-1][2] * 1e3))
    a, b, _ = min(table, key=lambda r: r[2])
    if cache_path:
        cache[key] = dict(push_to_pull=a, pull_to_push=b, table=table)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return a, b, table
