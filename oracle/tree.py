"""Decision-tree kernel choice with the paper's "unknown prediction" rule
(test infrastructure).

A fitted binary tree is walked from the root: at an inner node holding
(feature f, threshold t) the walk goes left when x[f] <= t.  A leaf's class
is the majority of its bucket (Section II-A).  When the majority is not unique
(a tie) the prediction is "unknown": level N then repeats the choice made for
level N-1, and at the first level the edge-centric kernel is used, the one
least likely to be very slow (Section IV-A, unknown-prediction paragraphs).

scikit-learn compares features stored as float32 against float64
thresholds, so the walk converts each feature to float32 first.
"""
from __future__ import annotations

import numpy as np


def leaf_of(tree: dict, x) -> int:
    left, right = tree["left"], tree["right"]
    feat, thr = tree["feature"], tree["threshold"]
    node = 0
    while left[node] != -1:
        xv = float(np.float32(x[feat[node]]))
        node = left[node] if xv <= thr[node] else right[node]
    return node


def predict(tree: dict, x, prev_kernel: int, level: int, default_kernel: int):
    """Returns ``(kernel_id, unknown)`` for feature vector ``x`` at ``level``."""
    node = leaf_of(tree, x)
    counts = np.asarray(tree["value"][node], dtype=np.float64)
    top = counts.max()
    winners = np.flatnonzero(counts == top)
    if winners.shape[0] == 1:
        return int(tree["class_kernel"][int(winners[0])]), False
    return (int(prev_kernel) if level > 0 else int(default_kernel)), True
