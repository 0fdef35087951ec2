"""Oracle for the decision graph (Section 2.1): the <rho, delta> pairs that a user
reads to choose rho_min and delta_min, summarised as

* the top-k points by dependent distance among the non-noise points (rho >= rho_min),
  ordered by delta descending, then id ascending;
* a two-dimensional histogram of <rho, delta> over caller-given bin edges;
* a suggested delta_min: the largest ratio gap in the top-k list (the paper asks for a
  delta_min that singles out the points whose dependent distance is much longer than
  the others', after Def. 5).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.

Readings (also in the design notes):

* ties in delta go to the smaller id, as in the rank order of the exact method;
* histogram bins are half-open [e_i, e_{i+1}) except the last, which also holds its
  right edge (so an edge of +inf takes the densest point's infinite delta); values
  outside all bins are not counted;
* the suggestion looks at consecutive pairs (delta_j, delta_{j+1}) of the top list
  where delta_j is finite and above d_cut (a valid delta_min must exceed d_cut); it
  takes the pair with the largest ratio delta_j / delta_{j+1} (a zero delta_{j+1}
  makes it infinite; ties: the first pair) and suggests delta_min = delta_j, which
  makes the points of the list down to j centers (with the points of infinite
  delta).  No such pair: no suggestion.
"""
from __future__ import annotations

import math

import numpy as np


def top_delta(rho, delta, rho_min: int, k: int):
    """Ids, deltas and rhos of the k non-noise points of largest delta (ties: smaller id)."""
    rho = np.asarray(rho, np.int64)
    delta = np.asarray(delta, np.float64)
    ids = np.nonzero(rho >= rho_min)[0]
    order = np.lexsort((ids, -delta[ids]))  # delta descending, then id ascending
    sel = ids[order][:k]
    return sel.astype(np.int64), delta[sel], rho[sel]


def _bins(values, edges) -> np.ndarray:
    """Bin index of each value, -1 outside (half-open bins, the last one closed)."""
    edges = np.asarray(edges, np.float64)
    v = np.asarray(values, np.float64)
    nb = edges.size - 1
    i = np.searchsorted(edges, v, side="right") - 1
    i[(i == nb) & (v == edges[-1])] = nb - 1  # the last bin holds its right edge
    i[(i < 0) | (i >= nb)] = -1
    return i


def histogram(rho, delta, rho_edges, delta_edges) -> np.ndarray:
    """counts[i][j]: points with rho in rho bin i and delta in delta bin j."""
    nr, nd = len(rho_edges) - 1, len(delta_edges) - 1
    a = _bins(rho, rho_edges)
    b = _bins(delta, delta_edges)
    ok = (a >= 0) & (b >= 0)
    counts = np.zeros(nr * nd, np.int64)
    np.add.at(counts, a[ok] * nd + b[ok], 1)
    return counts.reshape(nr, nd)


def suggest_delta_min(top_deltas, d_cut: float):
    """(delta_min, centers among the list) or (None, 0) when no pair qualifies."""
    best, best_j = -1.0, -1
    t = [float(x) for x in top_deltas]
    for j in range(len(t) - 1):
        a, b = t[j], t[j + 1]
        if not (math.isfinite(a) and a > d_cut):
            continue
        ratio = math.inf if b == 0.0 else a / b
        if ratio > best:
            best, best_j = ratio, j
    if best_j < 0:
        return None, 0
    dmin = t[best_j]
    return dmin, sum(1 for x in t if x >= dmin)
