"""Per-level feature vector, written from its definition (test infrastructure).

The paper's candidate features (Section IV-A, feature list) are the graph size
(vertices and edges), the frontier size and the discovered-vertex count (each
absolute or as a fraction of the vertices), and a degree distribution given by
its five-number summary plus standard deviation.  Its best model (Section IV-B,
second paragraph) uses graph size, fraction discovered, the out-degree
distribution and the current frontier's vertex count.

Readings taken where the paper is silent:
  * edges = directed CSR entries (twice the undirected edge count);
  * quartiles use linear interpolation between order statistics (numpy's
    default), the standard deviation is the population one (ddof = 0);
  * on an undirected graph out-degree = in-degree = degree;
  * at level d (the step that expands the depth-d vertices) the frontier is
    the depth-d vertex count and "discovered" counts depths 0..d, over all
    vertices of the graph (not only the component).
"""
from __future__ import annotations

import numpy as np

NAMES = ("n_vertices", "n_edges", "deg_min", "deg_q1", "deg_median", "deg_q3", "deg_max",
         "deg_std", "frontier", "frontier_frac", "discovered", "discovered_frac")
N_FEATURES = len(NAMES)


def graph_features(offs) -> np.ndarray:
    offs = np.asarray(offs, dtype=np.int64)
    n = offs.shape[0] - 1
    deg = np.diff(offs).astype(np.float64)
    q1, med, q3 = np.percentile(deg, [25.0, 50.0, 75.0])
    return np.array([n, offs[-1], deg.min(), q1, med, q3, deg.max(), deg.std()], dtype=np.float64)


def level_features(offs, hist, d: int, gfeat=None) -> np.ndarray:
    """Feature vector for level d given the per-depth vertex counts ``hist``."""
    gf = graph_features(offs) if gfeat is None else gfeat
    n = float(gf[0])
    nf = float(hist[d])
    disc = float(np.sum(np.asarray(hist[: d + 1], dtype=np.int64)))
    return np.concatenate([gf, [nf, nf / n, disc, disc / n]])
