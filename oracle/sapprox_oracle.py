"""Oracle for S-Approx-DPC (Section 5): one sampled point per cell of a finer
grid carries the cell, so point clustering becomes cell clustering.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
never does, and this module imports nothing from the product package.

Steps, in the section's order:

1. the grid G' of cells of side eps * d_cut / sqrt(d) (0 < eps <= 1), and one
   picked point per cell;
2. the exact local density of each picked point (Def. 1, against all points), and
   N(c): the cells other than c holding a point strictly within d_cut of c's pick;
3. dependent points: a point that was not picked takes its cell's pick; a pick p_i
   takes, in the first phase, a pick of higher density in a cell of N(c), and in
   the second phase (no such pick) its nearest pick of higher density (the
   temporary clusters of the section only prune that search, so they are not
   needed to define its result);
4. labels (Defs. 4-6).  A point that was not picked has no density of its own: it
   reports its pick's density and joins its pick's cluster (the section leaves
   rho_min out for it).

Readings where the section leaves a choice (each is also in the design notes):

* integer coordinates: the cell side is Le = 1 + floor(sqrt((Re - 1) / d)) with
  Re = ceil(e^2), e = eps * d_cut as a double product, so two points of one cell
  lie strictly within e; the cell of a point is (x_1 // Le, ..., x_d // Le);
* the pick of a cell is its smallest id;
* "higher local density" is the exact method's rank order (rho descending, id
  ascending) over the picks;
* the first phase takes, among the qualifying picks of the cells of N(c), the
  nearest (ties: smaller id); its dependent distance is the true distance, at most
  (1 + eps) d_cut;
* a point that was not picked gets dep = its pick and delta = the true distance to
  it (below eps * d_cut <= d_cut < delta_min, so it is never a center);
* the second phase returns the exact nearest higher-ranked pick and its distance.
"""
from __future__ import annotations

import math
import numpy as np

from . import dpc_oracle


def eps_cutoff_square(d_cut: float, eps: float) -> int:
    """Re = ceil(e^2) for e = eps * d_cut rounded to a double (one IEEE product),
    exact as for d_cut; 1 if the product underflows to zero."""
    e = float(eps) * float(d_cut)
    return dpc_oracle.cutoff_square(e) if e > 0.0 else 1


def cell_side(Re: int, d: int) -> int:
    return 1 + math.isqrt((Re - 1) // d)


def pick_of(ids) -> int:
    """The cell's picked point: its smallest id."""
    return min(ids)


def within(d2, R: int):
    """Strictly within d_cut (Def. 1's ball), on exact squared distances."""
    return d2 < R


def nearest(p, i: int, cands) -> tuple[int, int]:
    """(D2, id) of the candidate nearest to point i (ties: smaller id)."""
    return min((int(np.sum((p[i] - p[q]) ** 2)), int(q)) for q in cands)


def sapprox_dpc(pts, d_cut: float, eps: float, rho_min: int, delta_min: float) -> dict:
    if not (0.0 < eps <= 1.0):
        raise ValueError("eps must be in (0, 1]")
    p = np.asarray(pts, dtype=np.int64)
    n, d = p.shape
    R = dpc_oracle.cutoff_square(d_cut)
    Le = cell_side(eps_cutoff_square(d_cut, eps), d)
    cell = [tuple(int(v) for v in row) for row in (p // Le)]
    members: dict[tuple, list[int]] = {}
    for i, c in enumerate(cell):
        members.setdefault(c, []).append(i)
    pick = {c: pick_of(m) for c, m in members.items()}
    picks = np.array(sorted(pick.values()), dtype=np.int64)
    is_pick = np.zeros(n, dtype=bool)
    is_pick[picks] = True

    # step 2: exact densities of the picks, and N(c)
    rho_pick = {}
    near = {}
    for c, s in pick.items():
        d2 = np.sum((p - p[s]) ** 2, axis=1)
        inside = np.nonzero(within(d2, R))[0]
        rho_pick[s] = int(inside.size)
        near[c] = sorted({cell[j] for j in inside if cell[j] != c})
    prho = np.array([rho_pick[s] for s in picks], dtype=np.int64)
    order = np.lexsort((picks, -prho))  # rank order over the picks
    prank = np.empty(picks.size, dtype=np.int64)
    prank[order] = np.arange(picks.size)
    rank_of = {int(s): int(r) for s, r in zip(picks, prank)}

    rho = np.empty(n, dtype=np.int64)
    dep = np.full(n, -1, dtype=np.int64)
    delta = np.full(n, np.inf)
    phase = np.zeros(n, dtype=np.int8)  # 0 not picked, 1 first phase, 2 second phase
    for i in range(n):
        c = cell[i]
        s = pick[c]
        rho[i] = rho_pick[s]
        if i != s:
            dep[i] = s
            delta[i] = math.sqrt(float(np.sum((p[i] - p[s]) ** 2)))
            continue
        # first phase: higher-ranked picks of the cells of N(c), the nearest
        cands = [pick[c2] for c2 in near[c] if rank_of[pick[c2]] < rank_of[i]]
        if cands:
            phase[i] = 1
        else:
            # second phase: the nearest higher-ranked pick of all
            cands = [int(q) for q in picks if rank_of[int(q)] < rank_of[i]]
            phase[i] = 2
        if cands:
            key = nearest(p, i, cands)
            dep[i] = key[1]
            delta[i] = math.sqrt(float(key[0]))
    lab, nc = dpc_oracle.labels(rho, dep, delta, rho_min, delta_min)
    return {"rho": rho, "dep": dep, "delta": delta, "label": lab, "ncenters": nc, "picked": is_pick,
            "phase": phase, "side": Le}
