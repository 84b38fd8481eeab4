"""Training data, tree fitting and export (Sections IV-A, IV-B and IV-D).

The paper measures every implementation at every BFS level of many graphs
and roots, labels each level with its fastest implementation, and fits a
scikit-learn CART classifier (Gini impurity) on a 70% random split, checking
it on the other 30%.  The tree is then exported to flat arrays for a C
lookup.  Here:

  collect  per (graph, source, level): the library's feature vector and the
           median time of every kernel (33: eleven base kernels in three
           frontier-count variants) from the same saved BFS state
           (gsw_bfs_profile); the BFS advances with the level's fastest kernel.
  fit      DecisionTreeClassifier(criterion="gini").  Hyper-parameters (depth,
           minimum leaf, row weights) are chosen by the total-time ratio on
           VALIDATION graphs -- graphs of their own, disjoint from the
           training graphs and from every evaluated workload (the smallest
           tree within 0.5% of the best); a 3-fold cross-validation over the
           training graphs grouped by graph is reported beside it.  The
           shipped tree is trained on the training graphs only.  The report
           gives the paper's random 70/30 row split, a held-out-graph split of
           the training graphs, the validation graphs, and Table II of the
           paper computed on the validation traversals (slowdown against the
           best-per-level traversal for the tree, the best fixed kernel per
           graph, and every kernel).  The model variants the paper names as
           future work are fitted on the same rows and reported beside it: a
           regression tree per kernel (predict each kernel's level time, take
           the smallest) and a random forest classifier.
  solo     per row, the level's time when the search runs it in a
           single-workgroup multi-level launch (small top-down levels): the
           push kernels' times on such rows are replaced by it before fitting,
           since the profile times every level as a launch of its own.
  export   JSON with the flat node arrays gsw_tree_load() reads.

Every graph here is a synthetic family member at its own seed; the graphs and
sources evaluated by the benchmark (R-MAT 22 seed 2, the sweep's grid, Chung-Lu
and Erdos-Renyi graphs) are never trained or validated on.  Their families
and sizes do appear at other seeds (R-MAT 22 seeds 200-203, a 2048 x 2048
grid seed 210, Chung-Lu 2^23 seed 220, Erdos-Renyi 2^22 seed 230): the tree
cannot extrapolate a feature such as the vertex count past the largest
graph it was trained on.

    python -m paper_1708_01159_amd.train collect --out rows.npz
    python -m paper_1708_01159_amd.train collect --set valid --out valid.npz
    python -m paper_1708_01159_amd.train solo --rows rows.npz --out rows.npz
    python -m paper_1708_01159_amd.train solo --set valid --rows valid.npz --out valid.npz
    python -m paper_1708_01159_amd.train fit --rows rows.npz --valid valid.npz --out trees/mi355x.json
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

from . import graphgen as gg
from . import gsw

FEATURES = gsw.FEATURE_NAMES


def _directed(make, keep: float, seed: int, name: str):
    """A random ``keep`` share of a symmetric graph's arcs: one-way and
    reciprocated arcs, so in-, out- and absolute degrees differ."""
    def build():
        g = make()
        rows = np.repeat(np.arange(g.n), g.degrees())
        m = np.random.default_rng(seed).random(g.nnz) < keep
        return gg.from_edges(g.n, rows[m], g.cols[m], symmetrize=False, name=name)
    return build


# (name, maker, sources) -- other seeds / sizes than the evaluated workloads
TRAIN_GRAPHS = [
    ("rmat16_s100", lambda: gg.rmat(16, 16, seed=100), 12),
    ("rmat18_s101", lambda: gg.rmat(18, 16, seed=101), 12),
    ("rmat20_s102", lambda: gg.rmat(20, 16, seed=102), 12),
    ("rmat21_ef8_s103", lambda: gg.rmat(21, 8, seed=103), 12),
    ("rmat19_ef32_s105", lambda: gg.rmat(19, 32, seed=105), 8),
    ("rmat20_flat_s106", lambda: gg.rmat(20, 16, 0.45, 0.22, 0.22, seed=106), 8),
    ("rmat22_s200", lambda: gg.rmat(22, 16, seed=200), 16),
    ("rmat22_s201", lambda: gg.rmat(22, 16, seed=201), 16),
    ("rmat22_s202", lambda: gg.rmat(22, 16, seed=202), 16),
    ("rmat22_s203", lambda: gg.rmat(22, 16, seed=203), 16),
    ("grid256_del5_s200", lambda: gg.grid(256, 256, 0.05, seed=200), 2),
    ("grid512x256_del2_s201", lambda: gg.grid(512, 256, 0.02, seed=201), 2),
    ("grid1024_del5_s202", lambda: gg.grid(1024, 1024, 0.05, seed=202), 1),
    ("grid2048_del5_s210", lambda: gg.grid(2048, 2048, 0.05, seed=210), 1),
    ("chunglu18_s300", lambda: gg.chung_lu(1 << 18, 2.1, 20.0, seed=300), 8),
    ("chunglu20_s301", lambda: gg.chung_lu(1 << 20, 2.1, 20.0, seed=301), 8),
    ("chunglu21_g25_s302", lambda: gg.chung_lu(1 << 21, 2.5, 10.0, seed=302), 8),
    ("chunglu22_s303", lambda: gg.chung_lu(1 << 22, 2.1, 20.0, seed=303), 8),
    ("chunglu23_s220", lambda: gg.chung_lu(1 << 23, 2.1, 20.0, seed=220), 6),
    ("er18_d8_s400", lambda: gg.erdos_renyi(1 << 18, 4 << 18, seed=400), 8),
    ("er20_d8_s401", lambda: gg.erdos_renyi(1 << 20, 4 << 20, seed=401), 8),
    ("er21_d4_s402", lambda: gg.erdos_renyi(1 << 21, 2 << 21, seed=402), 8),
    ("er20_d32_s403", lambda: gg.erdos_renyi(1 << 20, 16 << 20, seed=403), 8),
    ("er22_d8_s404", lambda: gg.erdos_renyi(1 << 22, 4 << 22, seed=404), 8),
    ("er22_d8_s230", lambda: gg.erdos_renyi(1 << 22, 4 << 22, seed=230), 6),
    ("rmat20_dir60_s500", _directed(lambda: gg.rmat(20, 16, seed=500), 0.6, 500, "rmat20_dir60_s500"), 8),
    ("chunglu20_dir50_s501", _directed(lambda: gg.chung_lu(1 << 20, 2.1, 20.0, seed=501), 0.5, 501,
                                       "chunglu20_dir50_s501"), 8),
]

# Validation graphs: hyper-parameters and model selection only (never trained on)
VALID_GRAPHS = [
    ("rmat21_s600", lambda: gg.rmat(21, 16, seed=600), 12),
    ("rmat22_s601", lambda: gg.rmat(22, 16, seed=601), 12),
    ("grid768_del5_s602", lambda: gg.grid(768, 768, 0.05, seed=602), 1),
    ("chunglu21_s603", lambda: gg.chung_lu(1 << 21, 2.1, 20.0, seed=603), 8),
    ("er21_d8_s604", lambda: gg.erdos_renyi(1 << 21, 4 << 21, seed=604), 8),
    ("rmat19_dir70_s605", _directed(lambda: gg.rmat(19, 16, seed=605), 0.7, 605, "rmat19_dir70_s605"), 8),
]


def collect(graphs=None, reps: int = 3, kernels=None, log=print, source_seed: int = 900):
    """Returns a dict of arrays: X [rows, F], T [rows, K], graph, source, level."""
    import torch  # noqa: F401  (one HIP runtime: torch's)

    ks = list(kernels if kernels is not None else range(gsw.N_KERNELS))
    X, T, gname, src, lvl = [], [], [], [], []
    for name, maker, nsrc in graphs or TRAIN_GRAPHS:
        t0 = time.time()
        g = maker()
        flags = gsw.TRUSTED | (0 if "_dir" in name else gsw.ASSUME_SYMMETRIC)
        G = gsw.Graph.from_csr(g.offs, g.cols, flags=flags)
        r = reps if g.n < (1 << 19) or "grid" not in name else max(1, reps - 1)
        for i, s in enumerate(gg.pick_sources(g, nsrc, source_seed)):
            times, fr, _ = gsw.bfs_profile(G, int(s), kernels=ks, reps=r, advance_kernel=-1)
            log("  %s source %d/%d: %d levels (%.1f s)" % (name, i + 1, nsrc, len(fr), time.time() - t0))
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


# A single-workgroup launch runs up to 32 small top-down levels back to back
# (gsw_bfs_opts.no_solo); the profile above times each level as one launch
# of its own, so on such levels it charges a push kernel a whole launch
# (about 6-12 us on MI355X) where the search pays a few microseconds.  The
# share of one launch's cost that each of its levels carries:
SOLO_LAUNCH_SHARE_MS = 0.0005


def solo_times(graphs, rows, log=print):
    """Per row: the device time (ms) of the row's level when the search runs
    it in a single-workgroup launch, NaN when it does not.  One search per
    (graph, source) with push_vertex at every level and device-stamped level
    times; BFS level sets do not depend on the kernel, so its level d is the
    row's level d, and every queue-driven top-down kernel runs such a level
    the same way."""
    import torch  # noqa: F401  (one HIP runtime: torch's)

    out = np.full(len(rows["level"]), np.nan)
    want = {}
    for i, (gname, s, d) in enumerate(zip(rows["graph"], rows["source"], rows["level"])):
        want.setdefault(str(gname), {}).setdefault(int(s), []).append((int(d), i))
    for name, maker, _ in graphs:
        if name not in want:
            continue
        t0 = time.time()
        g = maker()
        flags = gsw.TRUSTED | (0 if "_dir" in name else gsw.ASSUME_SYMMETRIC)
        G = gsw.Graph.from_csr(g.offs, g.cols, flags=flags)
        n_solo = 0
        for s, items in want[name].items():
            _, _, tr = gsw.bfs(G, [s], policy="fixed", kernel=gsw.PUSH_VERTEX, parents=False, time_levels=True,
                               trace_cap=max(d for d, _ in items) + 64)
            by_level = {t.level: t for t in tr}
            for d, i in items:
                t = by_level.get(d)
                if t is not None and t.flags & 4:
                    out[i] = t.ms
                    n_solo += 1
        G.close()
        log("solo times %-22s %d of %d rows (%.1f s)" % (name, n_solo, sum(len(v) for v in want[name].values()),
                                                        time.time() - t0))
    return out


def apply_solo(T, solo_ms, kernels):
    """T with the push kernels' times replaced, on rows whose level runs in a
    single-workgroup launch, by that launch's cost per level (the level's
    device time plus SOLO_LAUNCH_SHARE_MS)."""
    T = np.array(T, dtype=np.float64, copy=True)
    m = ~np.isnan(np.asarray(solo_ms, dtype=np.float64))
    cols = [j for j, k in enumerate(kernels) if gsw.kernel_base(int(k)) <= gsw.PUSH_EDGE]
    for j in cols:
        T[m, j] = np.asarray(solo_ms)[m] + SOLO_LAUNCH_SHARE_MS
    return T


TIE_TOL = 0.02  # level times within 2% of the fastest count as ties (measurement noise)


def labels(T, tol: float = TIE_TOL):
    """Fastest kernel index per row: the lowest index whose time is within
    `tol` of the row's fastest (ties go to the lowest index; unmeasured = -1
    ignored).  Kernels that run a level the same way -- every queue-driven
    push kernel when the level goes to one workgroup -- then get one label
    instead of whichever the noise favoured."""
    t = np.where(T < 0, np.inf, T)
    best = t.min(axis=1, keepdims=True)
    return np.argmax(t <= best * (1.0 + tol), axis=1)


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


def scores(chosen_col, T):
    """(accuracy, mean per-row slowdown, total-time ratio) of choosing column
    chosen_col[i] at row i."""
    t = np.where(T < 0, np.inf, T)
    best = t.min(axis=1)
    chosen = t[np.arange(len(t)), chosen_col]
    return (float(np.mean(chosen_col == labels(T))), float(np.mean(chosen / best)),
            float(chosen.sum() / best.sum()))


def relabel_leaves(clf, X, T):
    """Cost-sensitive leaves: each leaf of the fitted tree predicts the
    kernel, among the tree's classes, with the least total measured time over
    the training rows the leaf holds, instead of the most frequent label.
    The splits stay the Gini tree's.  A frontier's size and the discovered
    count cannot tell a hub from a leaf vertex, so rows that look alike can
    have very different costs per kernel: the majority label (the kernel
    that is a hair faster on most of them) may be very slow on the rest,
    while the least total time weighs every row by what the choice costs."""
    t = np.where(T < 0, np.inf, T)
    leaf = clf.apply(X.astype(np.float32))
    cls = clf.classes_.astype(np.int64)
    v = clf.tree_.value
    for nd in np.unique(leaf):
        tot = t[leaf == nd][:, cls].sum(axis=0)
        best = int(np.argmin(tot))
        w = float(v[nd].sum())
        v[nd] = 0.0
        v[nd, 0, best] = w if w > 0 else 1.0
    return clf


def tree_columns(clf, X):
    """Column (kernel index into the rows' kernel list) the classifier picks.
    Features are compared in float32, as the library does."""
    return clf.predict(X.astype(np.float32)).astype(np.int64)


def evaluate(clf, X, T):
    return scores(tree_columns(clf, X), T)


def family(graph_name: str) -> str:
    """The generator family of a training graph's name (its leading letters:
    rmat, er, grid, chunglu)."""
    m = re.match(r"[a-z]+", str(graph_name))
    return m.group(0) if m else str(graph_name)


def family_ratios(chosen_col, T, graph):
    """Total-time ratio (chosen over fastest) of choosing column chosen_col[i]
    at row i, per graph family: a tree can look fine pooled and still lose
    one family badly."""
    t = np.where(T < 0, np.inf, T)
    chosen = t[np.arange(len(t)), chosen_col]
    best = t.min(axis=1)
    fam = np.array([family(x) for x in graph])
    return {f: round(float(chosen[fam == f].sum() / best[fam == f].sum()), 4) for f in sorted(set(fam.tolist()))}


def _named(t):
    return dict(zip(("accuracy", "mean_slowdown", "time_ratio"), t))


def table2(cols_by_model, T, graph, source, names):
    """The paper's Table II on a set of traversals: for each model (a column
    choice per row) and for every kernel used at every level, the traversal's
    time over the best-per-level traversal's, summarised as the share of
    traversals at the optimum (within 0.1%), within 1-2x, above 5x and above
    20x, the mean and the worst; "best fixed" is the fastest single kernel of
    each graph (the paper's "Oracle")."""
    t = np.where(T < 0, np.inf, T)
    best = t.min(axis=1)
    keys = sorted(set(zip(graph.tolist(), source.tolist())))
    idx = {k: i for i, k in enumerate(keys)}
    trav = np.array([idx[(g, s)] for g, s in zip(graph.tolist(), source.tolist())])
    opt = np.bincount(trav, weights=best, minlength=len(keys))

    def summary(ratio):
        ratio = np.asarray(ratio)
        return {"optimal": round(float(np.mean(ratio <= 1.001)), 3),
                "1-2x": round(float(np.mean((ratio > 1.001) & (ratio <= 2.0))), 3),
                ">5x": round(float(np.mean(ratio > 5.0)), 3), ">20x": round(float(np.mean(ratio > 20.0)), 3),
                "average": round(float(np.mean(ratio)), 3), "worst": round(float(np.max(ratio)), 3)}

    out = {}
    for name, cols in cols_by_model.items():
        tt = np.bincount(trav, weights=t[np.arange(len(t)), cols], minlength=len(keys))
        out[name] = summary(tt / opt)
    per_k = {}
    for k in range(t.shape[1]):
        per_k[k] = np.bincount(trav, weights=t[:, k], minlength=len(keys)) / opt
    # best fixed kernel per graph
    gk = np.array([g for g, _ in keys])
    oracle = np.empty(len(keys))
    for gname in np.unique(gk):
        m = gk == gname
        tot = {k: np.sum(per_k[k][m] * opt[m]) for k in per_k}
        kb = min(tot, key=tot.get)
        oracle[m] = per_k[kb][m]
    out["best fixed kernel per graph"] = summary(oracle)
    for k in per_k:
        if np.all(np.isfinite(per_k[k])):
            out[names[k]] = summary(per_k[k])
    return out


def _model_variants(Xtr, Ttr, Xva, Tva, seed):
    """The paper's future-work models on the same rows: a regression tree per
    kernel (predict log level time, pick the smallest) and a random forest."""
    from sklearn.ensemble import RandomForestClassifier
    from sklearn.tree import DecisionTreeRegressor

    t = np.where(Ttr < 0, np.nan, Ttr)
    pred = np.full((len(Xva), Ttr.shape[1]), np.inf)
    for k in range(Ttr.shape[1]):
        ok = np.isfinite(t[:, k]) & (t[:, k] > 0)
        if ok.sum() < 10:
            continue
        reg = DecisionTreeRegressor(max_depth=10, min_samples_leaf=5, random_state=seed)
        reg.fit(Xtr[ok].astype(np.float32), np.log(t[ok, k]))
        pred[:, k] = reg.predict(Xva.astype(np.float32))
    reg_cols = np.argmin(pred, axis=1)
    rf = RandomForestClassifier(n_estimators=64, max_depth=12, min_samples_leaf=5, random_state=seed, n_jobs=-1)
    rf.fit(Xtr.astype(np.float32), labels(Ttr))
    rf_cols = rf.predict(Xva.astype(np.float32)).astype(np.int64)
    return reg_cols, rf_cols


SELECT_TOL = 0.005


def _graph_folds(graph, k: int, seed: int):
    """k boolean row masks, each holding the rows of about 1/k of the graphs."""
    names = np.unique(graph)
    order = np.random.default_rng(seed).permutation(len(names))
    return [np.isin(graph, names[order[i::k]]) for i in range(k)]


GRID = [(d, leaf, w, lv) for d in (6, 8, 10, 12) for leaf in (1, 5, 20) for w in ("none", "regret")
        for lv in ("majority", "time")]


def fit(rows, valid, seed=0, log=print, grid=GRID):
    from sklearn.tree import DecisionTreeClassifier

    X, T, graph, source = rows["X"], rows["T"], rows["graph"], rows["source"]
    Xv, Tv, gv, sv = valid["X"], valid["T"], valid["graph"], valid["source"]
    ks = [int(k) for k in rows["kernels"]]
    assert [int(k) for k in valid["kernels"]] == ks
    y = labels(T)

    def make(depth, leaf):
        return DecisionTreeClassifier(criterion="gini", max_depth=depth, min_samples_leaf=leaf, random_state=seed)

    def fit_one(depth, leaf, leaves, Xf, yf, Tf, wf):
        c = make(depth, leaf).fit(Xf, yf, sample_weight=wf)
        return relabel_leaves(c, Xf, Tf) if leaves == "time" else c

    # hyper-parameters by the validation graphs' total-time ratio: the
    # smallest tree within SELECT_TOL of the best; the 3-fold cross-validation
    # over the training graphs grouped by graph (each fold's graphs predicted
    # by a tree fitted on the others) is reported beside it
    folds = _graph_folds(graph, 3, seed)
    sel = []
    for depth, leaf, wscheme, leaves in grid:
        w = _weights(T, graph, wscheme)
        clf = fit_one(depth, leaf, leaves, X, y, T, w)
        acc, slow, ratio = evaluate(clf, Xv, Tv)
        cols = np.zeros(len(y), dtype=np.int64)
        for f in folds:
            c = fit_one(depth, leaf, leaves, X[~f], y[~f], T[~f], None if w is None else w[~f])
            cols[f] = tree_columns(c, X[f])
        cv = scores(cols, T)[2]
        sel.append(dict(max_depth=depth, min_samples_leaf=leaf, weights=wscheme, leaves=leaves,
                        valid_time_ratio=round(ratio, 4), valid_accuracy=round(acc, 4),
                        graph_cv_time_ratio=round(cv, 4), nodes=int(clf.tree_.node_count)))
        log("depth %2d leaf %2d %-6s %-8s: validation time ratio %.4f, accuracy %.3f; grouped CV %.4f; %d nodes"
            % (depth, leaf, wscheme, leaves, ratio, acc, cv, clf.tree_.node_count))
    top = min(r["valid_time_ratio"] for r in sel)
    best = min((r for r in sel if r["valid_time_ratio"] <= top * (1.0 + SELECT_TOL)),
               key=lambda r: (r["nodes"], r["graph_cv_time_ratio"], r["valid_time_ratio"]))
    depth, leaf, wscheme, leaves = best["max_depth"], best["min_samples_leaf"], best["weights"], best["leaves"]
    w = _weights(T, graph, wscheme)
    final = fit_one(depth, leaf, leaves, X, y, T, w)
    report = {"selection": {"chosen": best, "grid": sel,
                            "by": "validation graphs' total-time ratio: the smallest tree within %.1f%% of the best "
                                  "(equal sizes: the better graph-grouped cross-validation)" % (100 * SELECT_TOL)}}
    rng = np.random.default_rng(seed)
    # the paper's split: 70% of the training rows at random
    perm = rng.permutation(len(y))
    cut = int(0.7 * len(y))
    tr, te = perm[:cut], perm[cut:]
    c1 = fit_one(depth, leaf, leaves, X[tr], y[tr], T[tr], None if w is None else w[tr])
    report["row_split"] = _named(evaluate(c1, X[te], T[te]))
    # held-out training graphs: every graph predicted by a tree fitted on the
    # other folds (3 folds grouped by graph), and one 70/30 split by graph
    cols = np.zeros(len(y), dtype=np.int64)
    for f in folds:
        c = fit_one(depth, leaf, leaves, X[~f], y[~f], T[~f], None if w is None else w[~f])
        cols[f] = tree_columns(c, X[f])
    report["graph_split"] = dict(_named(scores(cols, T)), folds=[sorted(np.unique(graph[f]).tolist()) for f in folds],
                                 by_family=family_ratios(cols, T, graph))
    names = np.unique(graph)
    hold = rng.choice(names, size=max(1, len(names) * 3 // 10), replace=False)
    m = np.isin(graph, hold)
    c2 = fit_one(depth, leaf, leaves, X[~m], y[~m], T[~m], None if w is None else w[~m])
    report["graph_split_one_30pct"] = dict(_named(evaluate(c2, X[m], T[m])), held_out=sorted(hold.tolist()))
    report["validation"] = dict(_named(evaluate(final, Xv, Tv)), graphs=sorted(np.unique(gv).tolist()),
                                by_family=family_ratios(tree_columns(final, Xv), Tv, gv))
    report["train_all"] = _named(evaluate(final, X, T))
    reg_cols, rf_cols = _model_variants(X, T, Xv, Tv, seed)
    report["model_variants_on_validation"] = {
        "classification tree (shipped)": report["validation"],
        "regression tree per kernel, argmin": _named(scores(reg_cols, Tv)),
        "random forest (64 trees)": _named(scores(rf_cols, Tv)),
    }
    report["table2_validation"] = table2(
        {"decision tree": tree_columns(final, Xv), "regression trees": reg_cols, "random forest": rf_cols},
        Tv, gv, sv, [gsw.KERNEL_NAMES[k] for k in ks])
    report["gini_importance"] = {FEATURES[i]: round(float(v), 4)
                                 for i, v in enumerate(final.feature_importances_) if v > 0}
    report["nodes"] = int(final.tree_.node_count)
    report["params"] = dict(max_depth=depth, min_samples_leaf=leaf, weights=wscheme, leaves=leaves, seed=seed,
                            rows=int(len(y)), valid_rows=int(len(Tv)))
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


def _load_rows(paths):
    """Rows of one or more collect files; where every file carries the solo
    pass (solo_ms), T is corrected with it (apply_solo)."""
    parts = [dict(np.load(p, allow_pickle=False)) for p in paths]
    rows = {k: np.concatenate([p[k] for p in parts]) for k in ("X", "T", "graph", "source", "level")}
    rows["kernels"] = parts[0]["kernels"]
    if all("solo_ms" in p for p in parts):
        rows["solo_ms"] = np.concatenate([p["solo_ms"] for p in parts])
        rows["T"] = apply_solo(rows["T"], rows["solo_ms"], rows["kernels"])
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1708_01159_amd.train")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--set", default="train", choices=["train", "valid"])
    c.add_argument("--reps", type=int, default=3)
    c.add_argument("--only", default=None, help="comma-separated graph names")
    so = sub.add_parser("solo", help="add the single-workgroup level times to a collect file")
    so.add_argument("--rows", required=True)
    so.add_argument("--set", default="train", choices=["train", "valid"])
    so.add_argument("--out", required=True)
    f = sub.add_parser("fit")
    f.add_argument("--rows", required=True, nargs="+")
    f.add_argument("--valid", required=True, nargs="+")
    f.add_argument("--out", required=True)
    f.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    if a.cmd == "solo":
        rows = dict(np.load(a.rows, allow_pickle=False))
        rows["solo_ms"] = solo_times(TRAIN_GRAPHS if a.set == "train" else VALID_GRAPHS, rows,
                                     log=lambda *x: print(*x, flush=True))
        np.savez_compressed(a.out, **rows)
        print("wrote", a.out, int(np.sum(~np.isnan(rows["solo_ms"]))), "solo rows of", len(rows["level"]), flush=True)
        return
    if a.cmd == "collect":
        graphs = TRAIN_GRAPHS if a.set == "train" else VALID_GRAPHS
        if a.only:
            want = set(a.only.split(","))
            graphs = [x for x in graphs if x[0] in want]
        rows = collect(graphs, reps=a.reps, log=lambda *x: print(*x, flush=True))
        np.savez_compressed(a.out, **rows)
        print("wrote", a.out, len(rows["X"]), "rows", flush=True)
    else:
        clf, ks, report = fit(_load_rows(a.rows), _load_rows(a.valid), a.seed,
                              log=lambda *x: print(*x, file=sys.stderr, flush=True))
        export(clf, ks, a.out, report)
        print(json.dumps({k: v for k, v in report.items() if k not in ("selection", "table2_validation")}, indent=1))


if __name__ == "__main__":
    main()
