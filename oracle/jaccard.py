"""Oracle of JaccardWithWindows -- TEST INFRASTRUCTURE ONLY.

Plain Python over sets, for small graphs, following the algorithm of the
section "Increasing Compression Ratio" step by step: the vertex ids are cut
into windows of `window` consecutive ids; inside a window, slice sets of
`sigma` positions are filled in order. Each set starts from the unassigned
column of highest degree; the set's row union R is that column's neighbour
set. Each further position takes, among the unassigned columns sharing at
least one row with R, the one maximising
    inter / (|R| + deg - inter),   inter = |nbrs(column) and R|,
which is the Jaccard similarity (the equation of that section) between the
column's neighbour set and R; if no column shares a row with R, the
highest-degree unassigned column is taken instead. R grows by the chosen
column's neighbours.

inter is recomputed from its definition for every candidate (the paper's
incremental update of inter is an optimisation of the same quantity).
Readings (the paper does not fix them): ties of either maximisation go to
the smaller id; the ratio is compared exactly (fractions); a window whose
width is not a multiple of sigma ends with a partial slice set; the graph is
undirected, so the neighbours through A and through its transpose coincide.

Returns new_of_old: position of every vertex (the algorithm's inverse
permutation).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def jaccard_with_windows(rp, col, sigma: int, window: int) -> np.ndarray:
    rp = np.asarray(rp, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = rp.size - 1
    nbrs = [frozenset(col[rp[j]:rp[j + 1]].tolist()) for j in range(n)]
    deg = [len(x) for x in nbrs]
    new_of_old = np.full(n, -1, dtype=np.int64)
    for ws in range(0, n, window):
        we = min(ws + window, n)
        unassigned = set(range(ws, we))

        def highest():
            return min(unassigned, key=lambda j: (-deg[j], j))

        for ss in range(ws, we, sigma):
            se = min(ss + sigma, we)
            j = highest()
            unassigned.discard(j)
            new_of_old[j] = ss
            r = set(nbrs[j])
            for pos in range(ss + 1, se):
                cands = [c for c in unassigned if nbrs[c] & r]
                if not cands:
                    j = highest()
                else:
                    def score(c):
                        inter = len(nbrs[c] & r)
                        return (Fraction(inter, len(r) + deg[c] - inter), -c)
                    j = max(cands, key=score)
                unassigned.discard(j)
                new_of_old[j] = pos
                r |= nbrs[j]
    return new_of_old


def count_slices(rp, col, new_of_old, sigma: int) -> int:
    """Slices of the BVSS after relabelling: for every slice set, the number
    of distinct rows adjacent to at least one of its sigma columns (Section
    BVSS: a slice exists for each such row)."""
    rp = np.asarray(rp, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nof = np.asarray(new_of_old, dtype=np.int64)
    src = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    key = (nof[src] // sigma) * (rp.size + 1) + nof[col]
    return int(np.unique(key).size)
