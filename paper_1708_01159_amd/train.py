"""Training data, tree fitting and export (Sections IV-A and IV-D).

The paper measures every implementation at every BFS level of many graphs
and roots, labels each level with its fastest implementation, and fits a
scikit-learn CART classifier (Gini impurity) on a 70% random split, checking
it on the other 30%.  The tree is then exported to flat arrays for a C
lookup.  Here:

  collect  per (graph, source, level): the library's feature vector and the
           median time of every kernel from the same saved BFS state
           (gsw_bfs_profile); the BFS advances with the level's fastest kernel.
  fit      DecisionTreeClassifier(criterion="gini") on the rows, with the
           paper's random 70/30 row split and, as a harder check, a split
           that holds out whole graphs; reports accuracy, the mean slowdown of
           the predicted kernel against the fastest one, and Gini importance.
  export   JSON with the flat node arrays gsw_tree_create() takes.

Workloads for training are synthetic graphs of the evaluated families at
other seeds and sizes; the graphs and sources evaluated by the benchmark are
never trained on.

    python -m paper_1708_01159_amd.train collect --out rows.npz
    python -m paper_1708_01159_amd.train fit --rows rows.npz --out trees/mi355x.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import graphgen as gg
from . import gsw

FEATURES = gsw.FEATURE_NAMES

# (name, maker, sources) -- other seeds / sizes than the evaluated workloads
TRAIN_GRAPHS = [
    ("rmat16_s100", lambda: gg.rmat(16, 16, seed=100), 12),
    ("rmat18_s101", lambda: gg.rmat(18, 16, seed=101), 12),
    ("rmat20_s102", lambda: gg.rmat(20, 16, seed=102), 16),
    ("rmat21_ef8_s103", lambda: gg.rmat(21, 8, seed=103), 16),
    ("rmat21_s104", lambda: gg.rmat(21, 16, seed=104), 16),
    ("rmat19_ef32_s105", lambda: gg.rmat(19, 32, seed=105), 12),
    ("rmat20_flat_s106", lambda: gg.rmat(20, 16, 0.45, 0.22, 0.22, seed=106), 12),
    ("grid256_del5_s200", lambda: gg.grid(256, 256, 0.05, seed=200), 3),
    ("grid512x256_del2_s201", lambda: gg.grid(512, 256, 0.02, seed=201), 2),
    ("grid1024_del5_s202", lambda: gg.grid(1024, 1024, 0.05, seed=202), 2),
    ("chunglu18_s300", lambda: gg.chung_lu(1 << 18, 2.1, 20.0, seed=300), 12),
    ("chunglu20_s301", lambda: gg.chung_lu(1 << 20, 2.1, 20.0, seed=301), 12),
    ("chunglu21_g25_s302", lambda: gg.chung_lu(1 << 21, 2.5, 10.0, seed=302), 12),
    ("er18_d8_s400", lambda: gg.erdos_renyi(1 << 18, 4 << 18, seed=400), 16),
    ("er20_d8_s401", lambda: gg.erdos_renyi(1 << 20, 4 << 20, seed=401), 16),
    ("er21_d4_s402", lambda: gg.erdos_renyi(1 << 21, 2 << 21, seed=402), 16),
    ("er20_d32_s403", lambda: gg.erdos_renyi(1 << 20, 16 << 20, seed=403), 16),
    # the evaluated sizes, at other seeds
    ("rmat22_s200", lambda: gg.rmat(22, 16, seed=200), 32),
    ("rmat22_s201", lambda: gg.rmat(22, 16, seed=201), 32),
    ("rmat22_s202", lambda: gg.rmat(22, 16, seed=202), 32),
    ("grid2048_del5_s210", lambda: gg.grid(2048, 2048, 0.05, seed=210), 2),
    ("chunglu23_s220", lambda: gg.chung_lu(1 << 23, 2.1, 20.0, seed=220), 16),
    ("er22_d8_s230", lambda: gg.erdos_renyi(1 << 22, 4 << 22, seed=230), 24),
]


def collect(graphs=None, reps: int = 3, kernels=None, log=print, source_seed: int = 900):
    """Returns a dict of arrays: X [rows, F], T [rows, K], graph, source, level."""
    import torch  # noqa: F401  (one HIP runtime: torch's)

    ks = list(kernels if kernels is not None else range(gsw.N_KERNELS))
    X, T, gname, src, lvl = [], [], [], [], []
    for name, maker, nsrc in graphs or TRAIN_GRAPHS:
        t0 = time.time()
        g = maker()
        G = gsw.Graph.from_csr(g.offs, g.cols, flags=gsw.ASSUME_SYMMETRIC | gsw.TRUSTED)
        for s in gg.pick_sources(g, nsrc, source_seed):
            times, fr, _ = gsw.bfs_profile(G, int(s), kernels=ks, reps=reps, advance_kernel=-1)
            disc = np.cumsum(fr)
            for d in range(len(fr)):
                X.append(G.level_features(int(fr[d]), int(disc[d])))
                T.append(times[d])
                gname.append(name)
                src.append(int(s))
                lvl.append(d)
        G.close()
        log("collected %-22s n=%-9d nnz=%-10d rows=%d (%.1f s)" % (name, g.n, g.nnz, len(X), time.time() - t0))
    return dict(X=np.array(X), T=np.array(T, dtype=np.float64), graph=np.array(gname),
                source=np.array(src), level=np.array(lvl), kernels=np.array(ks))


def labels(T):
    """Fastest kernel index per row (ties -> lowest index; unmeasured = -1 ignored)."""
    t = np.where(T < 0, np.inf, T)
    return np.argmin(t, axis=1)


def _weights(T, graph, scheme: str):
    if scheme == "none":
        return None
    t = np.where(T < 0, np.nan, T)
    if scheme == "regret":  # cost of a wrong choice at this level
        w = np.nanmedian(t, axis=1) - np.nanmin(t, axis=1) + 1e-4
        return w / w.mean()
    if scheme == "graph":  # every graph weighs the same
        w = np.ones(len(graph))
        for gname in np.unique(graph):
            m = graph == gname
            w[m] = 1.0 / m.sum()
        return w / w.mean()
    raise ValueError(scheme)


def evaluate(clf, X, T, ks):
    """(accuracy, mean slowdown of predicted/fastest per row, total-time ratio)."""
    t = np.where(T < 0, np.inf, T)
    best = t.min(axis=1)
    pred = clf.predict(X.astype(np.float32))
    col = np.searchsorted(clf.classes_, pred)
    chosen = t[np.arange(len(t)), clf.classes_[col]]
    acc = float(np.mean(clf.classes_[col] == labels(T)))
    return acc, float(np.mean(chosen / best)), float(chosen.sum() / best.sum())


def fit(rows, max_depth=8, min_samples_leaf=5, weights="regret", seed=0, log=print):
    from sklearn.tree import DecisionTreeClassifier

    X, T, graph = rows["X"], rows["T"], rows["graph"]
    ks = [int(k) for k in rows["kernels"]]
    y = labels(T)
    rng = np.random.default_rng(seed)
    # the paper's split: 70% of rows at random
    perm = rng.permutation(len(y))
    cut = int(0.7 * len(y))
    tr, te = perm[:cut], perm[cut:]
    report = {}
    w = _weights(T, graph, weights)

    def make():
        return DecisionTreeClassifier(criterion="gini", max_depth=max_depth,
                                      min_samples_leaf=min_samples_leaf, random_state=seed)

    clf = make().fit(X[tr], y[tr], sample_weight=None if w is None else w[tr])
    report["row_split"] = dict(zip(("accuracy", "mean_slowdown", "time_ratio"),
                                   evaluate(clf, X[te], T[te], ks)))
    # held-out graphs
    names = np.unique(graph)
    hold = rng.choice(names, size=max(1, len(names) * 3 // 10), replace=False)
    m = np.isin(graph, hold)
    if (~m).sum() and m.sum():
        c2 = make().fit(X[~m], y[~m], sample_weight=None if w is None else w[~m])
        report["graph_split"] = dict(zip(("accuracy", "mean_slowdown", "time_ratio"),
                                         evaluate(c2, X[m], T[m], ks)), held_out=sorted(hold.tolist()))
    # final tree on every row
    final = make().fit(X, y, sample_weight=w)
    report["train_all"] = dict(zip(("accuracy", "mean_slowdown", "time_ratio"), evaluate(final, X, T, ks)))
    report["gini_importance"] = {FEATURES[i]: round(float(v), 4)
                                 for i, v in enumerate(final.feature_importances_) if v > 0}
    report["nodes"] = int(final.tree_.node_count)
    report["params"] = dict(max_depth=max_depth, min_samples_leaf=min_samples_leaf, weights=weights,
                            seed=seed, rows=int(len(y)))
    return final, ks, report


def export(clf, ks, path: str, report=None, name="mi355x"):
    t = clf.tree_
    arrays = dict(
        name=name,
        description="CART (Gini) tree over per-level features, trained on per-level kernel "
                    "times measured on MI355X.",
        feature_names=list(FEATURES),
        feature=[int(f) for f in t.feature],
        threshold=[float(x) for x in t.threshold],
        left=[int(c) for c in t.children_left],
        right=[int(c) for c in t.children_right],
        value=[[float(x) for x in v[0]] for v in t.value],
        class_kernel=[ks[int(c)] for c in clf.classes_],
        class_names=[gsw.KERNEL_NAMES[ks[int(c)]] for c in clf.classes_],
        report=report or {},
    )
    with open(path, "w") as f:
        json.dump(arrays, f, indent=1)
    return arrays


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1708_01159_amd.train")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--only", default=None, help="comma-separated graph names")
    f = sub.add_parser("fit")
    f.add_argument("--rows", required=True, nargs="+")
    f.add_argument("--out", required=True)
    f.add_argument("--max-depth", type=int, default=8)
    f.add_argument("--min-samples-leaf", type=int, default=5)
    f.add_argument("--weights", default="regret", choices=["none", "regret", "graph"])
    f.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        graphs = TRAIN_GRAPHS
        if a.only:
            want = set(a.only.split(","))
            graphs = [x for x in TRAIN_GRAPHS if x[0] in want]
        rows = collect(graphs, reps=a.reps, log=lambda *x: print(*x, flush=True))
        np.savez_compressed(a.out, **rows)
        print("wrote", a.out, len(rows["X"]), "rows", flush=True)
    else:
        parts = [dict(np.load(p, allow_pickle=False)) for p in a.rows]
        rows = {k: np.concatenate([p[k] for p in parts]) for k in ("X", "T", "graph", "source", "level")}
        rows["kernels"] = parts[0]["kernels"]
        clf, ks, report = fit(rows, a.max_depth, a.min_samples_leaf, a.weights, a.seed)
        export(clf, ks, a.out, report)
        print(json.dumps(report, indent=1))


if __name__ == "__main__":
    main()
