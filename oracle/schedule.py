"""Best-per-level ("optimal traversal") arithmetic (test infrastructure).

The paper's reference point is the traversal that uses the fastest kernel at
every level; its runtime is the sum of the per-level minima (Section IV-B,
first paragraph).  The best fixed kernel is the fastest non-switching one
(Section IV-B, definition of its "Oracle" row).  Ties between measured times
go to the lowest kernel id.
"""
from __future__ import annotations

import numpy as np


def best_per_level(times):
    """``times[level][kernel]`` (NaN = not measured) -> (choice[level], total)."""
    t = np.asarray(times, dtype=np.float64)
    choice = np.nanargmin(t, axis=1)
    total = float(np.nansum(np.nanmin(t, axis=1)))
    return choice.astype(np.int32), total


def best_fixed(times):
    """-> (kernel, total) of the fastest single kernel used at every level."""
    t = np.asarray(times, dtype=np.float64)
    tot = np.sum(t, axis=0)  # NaN when a kernel misses a level
    tot = np.where(np.isnan(tot), np.inf, tot)
    k = int(np.argmin(tot))
    return k, float(tot[k])
