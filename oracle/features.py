"""Per-level feature vector, written from its definition (test infrastructure).

The paper's candidate features (Section IV-A, feature list) are the graph size
(vertices and edges), the frontier size and the discovered-vertex count (each
absolute or as a fraction of the vertices), and the degree distribution, given
by the five-number summary plus standard deviation of the in-, out- or
absolute degrees.  Its best model (Section IV-B, second paragraph) uses graph
size, fraction discovered, the out-degree distribution and the current
frontier's vertex count.

Readings taken where the paper is silent:
  * edges = directed CSR entries (twice the undirected edge count);
  * quartiles use linear interpolation between order statistics (numpy's
    default), the standard deviation is the population one (ddof = 0);
  * out-degree of v = entries of row v; in-degree of v = entries equal to v
    over all rows; absolute degree of v = arcs entering or leaving v with an
    arc and its reverse counted once: out(v) + in(v) minus the entries u of
    row v for which the arc u -> v exists;
  * on a symmetric graph (every arc's reverse exists) the three
    distributions are the degree distribution;
  * at level d (the step that expands the depth-d vertices) the frontier is
    the depth-d vertex count and "discovered" counts depths 0..d, over all
    vertices of the graph (not only the component).
"""
from __future__ import annotations

import numpy as np

NAMES = ("n_vertices", "n_edges",
         "out_deg_min", "out_deg_q1", "out_deg_median", "out_deg_q3", "out_deg_max", "out_deg_std",
         "in_deg_min", "in_deg_q1", "in_deg_median", "in_deg_q3", "in_deg_max", "in_deg_std",
         "abs_deg_min", "abs_deg_q1", "abs_deg_median", "abs_deg_q3", "abs_deg_max", "abs_deg_std",
         "frontier", "frontier_frac", "discovered", "discovered_frac")
N_FEATURES = len(NAMES)
N_GRAPH_FEATURES = 20


def summary(deg) -> np.ndarray:
    """min, Q1, median, Q3, max, population std of a degree sequence."""
    deg = np.asarray(deg, dtype=np.float64)
    q1, med, q3 = np.percentile(deg, [25.0, 50.0, 75.0])
    return np.array([deg.min(), q1, med, q3, deg.max(), deg.std()], dtype=np.float64)


def _arcs(offs, cols):
    offs = np.asarray(offs, dtype=np.int64)
    rows = np.repeat(np.arange(offs.shape[0] - 1, dtype=np.int64), np.diff(offs))
    return rows, np.asarray(cols, dtype=np.int64)


def is_symmetric_set(offs, cols) -> bool:
    """Every arc (u, v) has its reverse (v, u); repeats do not matter."""
    rows, c = _arcs(offs, cols)
    n = np.asarray(offs).shape[0] - 1
    return set((rows * n + c).tolist()) == set((c * n + rows).tolist())


def degrees(offs, cols):
    """(out, in, absolute) degree of every vertex, from the definitions above."""
    offs = np.asarray(offs, dtype=np.int64)
    n = offs.shape[0] - 1
    out = np.diff(offs)
    if is_symmetric_set(offs, cols):
        return out, out.copy(), out.copy()
    rows, c = _arcs(offs, cols)
    indeg = np.bincount(c, minlength=n).astype(np.int64)
    arcset = set((rows * n + c).tolist())
    # entries u of row v whose reverse arc u -> v exists
    rev = np.array([int(u) * n + int(v) in arcset for v, u in zip(rows.tolist(), c.tolist())], dtype=bool)
    both = np.bincount(rows[rev], minlength=n).astype(np.int64)
    return out, indeg, out + indeg - both


def graph_features(offs, cols=None) -> np.ndarray:
    """Features 0..19.  Without ``cols`` the graph is taken as symmetric."""
    offs = np.asarray(offs, dtype=np.int64)
    n = offs.shape[0] - 1
    if cols is None:
        out = np.diff(offs)
        ind = ab = out
    else:
        out, ind, ab = degrees(offs, cols)
    return np.concatenate([[n, offs[-1]], summary(out), summary(ind), summary(ab)]).astype(np.float64)


def level_features(offs, hist, d: int, gfeat=None, cols=None) -> np.ndarray:
    """Feature vector for level d given the per-depth vertex counts ``hist``."""
    gf = graph_features(offs, cols) if gfeat is None else gfeat
    n = float(gf[0])
    nf = float(hist[d])
    disc = float(np.sum(np.asarray(hist[: d + 1], dtype=np.int64)))
    return np.concatenate([gf, [nf, nf / n, disc, disc / n]])
