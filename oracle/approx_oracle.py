"""Oracle for Approx-DPC (Section 4): exact local densities, approximate
dependent points where a higher-density point is known to lie within d_cut,
exact ones elsewhere.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
never does, and this module imports nothing from the product package.

The steps follow Section 4 in its order, with the exact method's readings
(``dpc_oracle``) for densities, ranks, exact dependent points and labels:

1. local density, exact (Section 4.2; Def. 1);
2. the grid G of cells of side d_cut / sqrt(d) (Section 4.1), and for each
   cell c: its points P(c), the point of maximum local density p*(c), the
   minimum local density min rho over P(c), and N(c), the cells other than c
   that hold a point closer than d_cut to p*(c);
3. approximate dependent points (Section 4.3): a point other than p*(c) takes
   p*(c); p*(c) itself takes p*(c') of a cell c' of N(c) whose minimum local
   density exceeds its own; either way the dependent distance is set to d_cut;
4. the exact dependent point and distance (Defs. 2-3) for every point left
   without one;
5. labels (Defs. 4-6) from these dependent points and distances.

Readings where the section leaves a choice (each is also listed in the design
notes):

* integer coordinates: the cell side is the integer L = 1 + floor(sqrt((R - 1)
  / d)), R = ceil(d_cut^2), so two points of one cell (coordinates differing by
  at most L - 1 in each dimension) have D2 <= d (L - 1)^2 <= R - 1 < R, i.e.
  lie strictly within d_cut, which is what the same-cell rule relies on; the
  cell of a point is (x_1 // L, ..., x_d // L);
* "maximum local density" ranks by (rho descending, id ascending), as the
  exact method's ties do;
* N(c) uses Def. 1's strict ball, D2 < R;
* among the cells of N(c) that qualify, the one with the smallest cell
  coordinates (compared as tuples, first dimension first) is taken;
* the approximate dependent distance is d_cut as a double.

Parity unpinned? No: tests pin it by Theorem 4 (the same centers as the exact
method, for delta_min > d_cut), a hand-worked example, and the invariants the
rules imply (see tests/test_approx_oracle.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import dpc_oracle


def cell_side(R: int, d: int) -> int:
    """L = 1 + floor(sqrt((R - 1) / d)): the largest integer side whose cells keep
    every pair of points strictly within d_cut."""
    return 1 + math.isqrt((R - 1) // d)


def cells_of(pts, L: int) -> list[tuple]:
    """The cell of each point: its coordinates floor-divided by L."""
    p = np.asarray(pts, dtype=np.int64)
    return [tuple(int(v) for v in row) for row in (p // L)]


def grid(pts, rho, R: int) -> dict:
    """Section 4.1's grid with the fields its cells keep (computed here in one
    pass after the densities): members, p*, min rho and N(c)."""
    p = np.asarray(pts, dtype=np.int64)
    n, d = p.shape
    L = cell_side(R, d)
    cell = cells_of(p, L)
    _, rank = dpc_oracle.density_order(rho)
    members: dict[tuple, list[int]] = {}
    for i, c in enumerate(cell):
        members.setdefault(c, []).append(i)
    pstar = {c: min(m, key=lambda i: rank[i]) for c, m in members.items()}
    minrho = {c: int(min(rho[i] for i in m)) for c, m in members.items()}
    near = {}
    for c, s in pstar.items():
        diff = p - p[s]
        d2 = np.sum(diff * diff, axis=1)
        near[c] = sorted({cell[j] for j in np.nonzero(d2 < R)[0] if cell[j] != c})
    return {"L": L, "cell": cell, "members": members, "pstar": pstar, "minrho": minrho, "near": near}


def approx_dependent(pts, rho, d_cut: float) -> dict:
    """Section 4.3: approximate dependent points where the rules allow, exact
    ones elsewhere.  Returns dep, delta and `approx` (True where the point's
    dependent point is approximate)."""
    p = np.asarray(pts, dtype=np.int64)
    n = p.shape[0]
    rho = np.asarray(rho, dtype=np.int64)
    R = dpc_oracle.cutoff_square(d_cut)
    g = grid(p, rho, R)
    dep = np.full(n, -1, dtype=np.int64)
    delta = np.full(n, np.inf)
    approx = np.zeros(n, dtype=bool)
    exact_ids = []
    for i in range(n):
        c = g["cell"][i]
        s = g["pstar"][c]
        if i != s:  # another point of the cell: p*(c), at most d_cut away
            dep[i], delta[i], approx[i] = s, float(d_cut), True
            continue
        qualify = [c2 for c2 in g["near"][c] if g["minrho"][c2] > rho[i]]
        if qualify:  # a nearby cell whose points all have a higher density
            dep[i], delta[i], approx[i] = g["pstar"][min(qualify)], float(d_cut), True
        else:
            exact_ids.append(i)
    if exact_ids:
        ex_dep, ex_d2 = dpc_oracle.dependent(p, rho)
        ex_delta = dpc_oracle.dependent_distance(ex_d2)
        for i in exact_ids:
            dep[i], delta[i] = ex_dep[i], ex_delta[i]
    return {"dep": dep, "delta": delta, "approx": approx, "grid": g}


def approx_dpc(pts, d_cut: float, rho_min: int, delta_min: float) -> dict:
    """The whole of Approx-DPC: exact rho, approximate dependents, labels."""
    rho = dpc_oracle.local_density(pts, d_cut)
    a = approx_dependent(pts, rho, d_cut)
    lab, nc = dpc_oracle.labels(rho, a["dep"], a["delta"], rho_min, delta_min)
    return {"rho": rho, "dep": a["dep"], "delta": a["delta"], "approx": a["approx"], "label": lab,
            "ncenters": nc, "grid": a["grid"]}
