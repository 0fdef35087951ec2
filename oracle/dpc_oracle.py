"""Oracle for exact density-peaks clustering: the plain O(n^2) method.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
never does, and this package imports nothing from the product package: the two
share no code.

It computes, slowly and in plain numpy with exact int64 arithmetic, what the
paper's straightforward algorithm computes (Section 2.2, "Straightforward
algorithm", steps 1-4), with the quantities of Definitions 1-6 (Section 2.1):

* local density (Def. 1, Eq. 1): the number of points of P strictly closer
  than d_cut, the point itself included;
* dependent point (Def. 2) and dependent distance (Def. 3): the nearest point
  among those of higher local density; the densest point has none and an
  infinite dependent distance;
* noise (Def. 4), cluster centers (Def. 5) and clusters (Def. 6).

Readings where the paper is silent or leaves a choice (each is also listed in
the design notes):

* squared distances are exact integers on integer coordinates, and
  ``dist < d_cut`` is decided as ``D2 < R`` with ``R = ceil(d_cut^2)`` computed
  exactly (rational arithmetic on the binary value of d_cut);
* "higher local density" is the strict order of (rho descending, id
  ascending): ties in rho, which Def. 2 breaks arbitrarily and Ex-DPC breaks by
  a random addend (Section 3), are broken by the smaller id;
* ties in distance go to the smaller id;
* the dependent distance is the correctly rounded FP64 square root of the
  exact squared distance, +inf for the densest point (dep = -1);
* the center test compares that FP64 value with delta_min as a double;
* noise points get label -1; other points get the id of their cluster center.

Every function here is pinned by tests that do not call it twice (hand-worked
example, independent brute force, scipy's kd-tree, closed forms, invariants).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

_INF_D2 = np.iinfo(np.int64).max


def cutoff_square(d_cut: float) -> int:
    """R = ceil(d_cut^2), exact.

    For an integer squared distance D2 >= 0: sqrt(D2) < d_cut  <=>  D2 < d_cut^2
    <=>  D2 < ceil(d_cut^2)  (Def. 1's strict inequality).
    """
    if not (isinstance(d_cut, (int, float)) and math.isfinite(d_cut) and d_cut > 0):
        raise ValueError("d_cut must be a finite positive number")
    f = Fraction(d_cut)
    return math.ceil(f * f)


def _as_points(pts) -> np.ndarray:
    p = np.asarray(pts)
    if p.ndim != 2:
        raise ValueError("points must be a 2-D array [n, d]")
    return p.astype(np.int64)


def squared_distances(p: np.ndarray, rows: slice, cols: np.ndarray | slice = slice(None)) -> np.ndarray:
    """Exact int64 squared Euclidean distances between p[rows] and p[cols]."""
    a = p[rows][:, None, :]
    b = p[cols][None, :, :]
    diff = a - b
    return np.sum(diff * diff, axis=2)


def local_density(pts, d_cut: float, block: int = 0) -> np.ndarray:
    """Def. 1 / Eq. 1, by a linear scan of P for every point (Scan step 1)."""
    p = _as_points(pts)
    n = p.shape[0]
    R = cutoff_square(d_cut)
    rho = np.empty(n, dtype=np.int64)
    if block <= 0:
        block = max(1, min(n, (1 << 23) // max(1, n * p.shape[1])))
    for s in range(0, n, block):
        rows = slice(s, min(n, s + block))
        rho[rows] = np.count_nonzero(squared_distances(p, rows) < R, axis=1)
    return rho


def density_order(rho) -> tuple[np.ndarray, np.ndarray]:
    """Scan step 2: sort P by descending local density (ties: smaller id first).

    Returns (order, rank): order[r] is the id at position r, rank is its inverse.
    """
    rho = np.asarray(rho, dtype=np.int64)
    ids = np.arange(rho.size)
    order = np.lexsort((ids, -rho))
    rank = np.empty(rho.size, dtype=np.int64)
    rank[order] = ids
    return order, rank


def dependent(pts, rho) -> tuple[np.ndarray, np.ndarray]:
    """Defs. 2-3 by Scan step 3: for each point, a linear scan of the density-
    sorted array that stops at the point itself (early termination).

    Returns (dep, d2): dep[i] is the dependent point's id (-1 for the densest
    point) and d2[i] the exact squared dependent distance (int64 max for it).
    Among equidistant candidates the smaller id wins.
    """
    p = _as_points(pts)
    n = p.shape[0]
    order, rank = density_order(rho)
    sorted_p = p[order]
    dep = np.full(n, -1, dtype=np.int64)
    d2 = np.full(n, _INF_D2, dtype=np.int64)
    for i in range(n):
        r = int(rank[i])
        if r == 0:
            continue
        diff = sorted_p[:r] - p[i]
        dist2 = np.sum(diff * diff, axis=1)
        best = dist2.min()
        dep[i] = order[:r][dist2 == best].min()
        d2[i] = best
    return dep, d2


def dependent_distance(d2) -> np.ndarray:
    """Def. 3: delta = dist(p_i, q_i) as the FP64 square root of the exact D2
    (D2 < 2^53, so the conversion to double is exact); +inf for the densest."""
    d2 = np.asarray(d2, dtype=np.int64)
    out = np.sqrt(d2.astype(np.float64))
    out[d2 == _INF_D2] = np.inf
    return out


def labels(rho, dep, delta, rho_min: int, delta_min: float) -> tuple[np.ndarray, int]:
    """Defs. 4-6 by Scan step 4: noise and centers, then depth-first label
    propagation from each center along the reverse dependency lists.

    A center's own dependent point is taken to be itself, so a center starts a
    cluster instead of joining its dependent point's.  Noise gets -1.
    Returns (label, number of centers).
    """
    rho = np.asarray(rho)
    dep = np.asarray(dep)
    delta = np.asarray(delta, dtype=np.float64)
    n = rho.size
    noise = rho < rho_min
    center = (~noise) & (delta >= float(delta_min))
    children: list[list[int]] = [[] for _ in range(n)]
    for i in range(n):
        if dep[i] >= 0:
            children[int(dep[i])].append(i)
    label = np.full(n, -1, dtype=np.int64)
    centers = np.nonzero(center)[0]
    for c in centers:
        c = int(c)
        label[c] = c
        stack = [c]
        while stack:
            u = stack.pop()
            for v in children[u]:
                if not noise[v] and not center[v]:
                    label[v] = c
                    stack.append(v)
    return label, int(centers.size)


def dpc(pts, d_cut: float, rho_min: int, delta_min: float) -> dict:
    """The whole plain method: rho, dependent point, delta, labels."""
    rho = local_density(pts, d_cut)
    dep, d2 = dependent(pts, rho)
    delta = dependent_distance(d2)
    lab, nc = labels(rho, dep, delta, rho_min, delta_min)
    return {"rho": rho, "dep": dep, "d2": d2, "delta": delta, "label": lab, "ncenters": nc}
