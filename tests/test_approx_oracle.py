"""Pins for the Approx-DPC oracle (Section 4), with no GPU.

What ties it to something other than itself:

* Theorem 4 (cluster center guarantee): for delta_min > d_cut the centers,
  and the noise, equal those of the exact method's oracle (itself pinned by
  brute force, a kd-tree and a hand-worked example);
* a hand-worked example (below), every value derived on paper;
* the approximation rules of Section 4.3 checked point by point with plain
  loops over the points (not the oracle's grid tables): a point other than its
  cell's densest takes that densest point, which lies strictly within d_cut;
  the densest point of a cell takes the densest point of a cell whose points
  all have a higher density and one of which lies strictly within d_cut;
  otherwise it keeps the exact dependent point and distance;
* the cell side: the largest integer side whose two farthest lattice points
  are still strictly within d_cut (checked with exact rationals).

The mutation tests plant plausible mistakes in the oracle and show that one of
these pins fails for each.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import approx_oracle, dpc_oracle
from paper_2207_04649_amd import inputs


def _cases():
    out = []
    for seed in range(4):
        for d in (1, 2, 3, 4):
            hi = [12, 60, 300][seed % 3]
            d_cut = [2.5, 4.0, 7.3, 11.0][(seed + d) % 4]
            out.append((inputs.uniform_points(160, d, hi, 500 + 10 * seed + d), d_cut))
    out.append((inputs.lattice_points(9, 2, 1), 3.0))     # D2 = R exactly on many pairs
    out.append((inputs.lattice_points(5, 3, 1), 2.0))
    out.append((inputs.lattice_points(12, 2, 2, 1), 4.0))
    job = inputs.blob_job(31, 400, 2, 4, 300.0, 900.0, 0.1)
    out.append((job.pts, job.d_cut))
    job = inputs.blob_job(32, 300, 3, 3, 300.0, 900.0, 0.1)
    out.append((job.pts, job.d_cut))
    out.append((inputs.uniform_points(200, 3, 6, 33), 1.5))     # R = 3 <= d: cells of side 1
    out.append((inputs.uniform_points(80, 8, 40, 34), 60.0))    # d = 8
    out.append((np.repeat(inputs.uniform_points(30, 2, 20, 35), 3, axis=0), 5.0))  # duplicates
    return out


def _rank(rho):
    return dpc_oracle.density_order(rho)[1]


# ---------------------------------------------------------------- pins

def pin_cell_side():
    for d in range(1, 9):
        for R in list(range(1, 120)) + [10 ** 6, 10 ** 6 + 1, 2 ** 40 - 1]:
            L = approx_oracle.cell_side(R, d)
            # The two farthest lattice points of a cell differ by L - 1 per axis;
            # with d_cut^2 just above R - 1 (any d_cut with ceil(d_cut^2) = R).
            dc2 = Fraction(R - 1) + Fraction(1, 2)
            assert L >= 1
            assert d * (L - 1) ** 2 < dc2, (d, R, L)
            assert d * L ** 2 >= R, (d, R, L)   # one more and the corners leave the ball


def pin_hand_example(impl):
    """Seven 2-D points, d_cut = 3 (R = 9, cell side 3):

    id: point   cell    rho  (neighbours with D2 < 9)
     0: (0,0)   (0,0)   3    1 (D2 2), 2 (4)
     1: (1,1)   (0,0)   3    0 (2), 2 (2)          [1-3: D2 = 9, outside]
     2: (2,0)   (0,0)   4    0, 1, 3 (5)
     3: (4,1)   (1,0)   3    2, 4 (2)              [3-6: D2 = 9, outside]
     4: (5,2)   (1,0)   3    3, 6 (5)
     5: (10,10) (3,3)   1
     6: (7,1)   (2,0)   2    4

    Rank order: 2, 0, 1, 3, 4, 6, 5.  p* of (0,0) is 2, of (1,0) is 3 (tie with 4,
    smaller id), of (2,0) is 6, of (3,3) is 5.  Min rho: 3, 3, 2, 1.
    0, 1 -> 2 and 4 -> 3 by the same-cell rule (delta = 3).
    6 is p*; its only neighbour 4 lies in (1,0) whose min rho 3 > 2 -> dep p*(1,0) = 3
    (delta = 3, though D2(6, 3) = 9: the dependent point need not be within d_cut).
    3 is p*; (0,0) holds 2 within d_cut but min rho 3 is not > 3 -> exact: among 2, 0,
    1 the nearest is 2 (D2 5) -> delta sqrt(5).
    2 is the densest -> no dependent point.  5 -> exact: nearest higher is 4 (D2 89).
    rho_min 2, delta_min 4: 5 is noise, 2 is the only center, everyone else joins it.
    """
    P = np.array([[0, 0], [1, 1], [2, 0], [4, 1], [5, 2], [10, 10], [7, 1]], np.int32)
    r = impl(P, 3.0, 2, 4.0)
    assert r["rho"].tolist() == [3, 3, 4, 3, 3, 1, 2]
    assert r["dep"].tolist() == [2, 2, -1, 2, 3, 4, 3]
    assert r["delta"].tolist() == [3.0, 3.0, float("inf"), 5 ** 0.5, 3.0, 89 ** 0.5, 3.0]
    assert r["approx"].tolist() == [True, True, False, False, True, False, True]
    assert r["label"].tolist() == [2, 2, 2, 2, 2, -1, 2]
    assert r["ncenters"] == 1


def pin_theorem4(impl, cases=None):
    for pts, d_cut in (cases or _cases()):
        ex = dpc_oracle.dpc(pts, d_cut, 1, 2 * d_cut)
        for rho_min in (1, 3):
            for delta_min in (float(np.nextafter(d_cut, np.inf)), 1.5 * d_cut, 3 * d_cut):
                exl, _ = dpc_oracle.labels(ex["rho"], ex["dep"], ex["delta"], rho_min, delta_min)
                r = impl(pts, d_cut, rho_min, delta_min)
                assert np.array_equal(r["rho"], ex["rho"])
                want = np.nonzero(exl == np.arange(exl.size))[0]
                got = np.nonzero(r["label"] == np.arange(exl.size))[0]
                assert np.array_equal(got, want), (d_cut, rho_min, delta_min)
                assert np.array_equal(r["label"] < 0, exl < 0)


def pin_rules(impl, cases=None):
    for pts, d_cut in (cases or _cases()):
        P = np.asarray(pts, np.int64)
        n, d = P.shape
        R = dpc_oracle.cutoff_square(d_cut)
        L = approx_oracle.cell_side(R, d)
        r = impl(P, d_cut, 1, 2 * d_cut)
        rho, dep, delta, approx = r["rho"], r["dep"], r["delta"], r["approx"]
        rank = _rank(rho)
        ex_dep, ex_d2 = dpc_oracle.dependent(P, rho)
        ex_delta = dpc_oracle.dependent_distance(ex_d2)
        cell = [tuple(int(v) // L for v in row) for row in P]
        in_cell = {}
        for i, c in enumerate(cell):
            in_cell.setdefault(c, []).append(i)
        top = {c: min(m, key=lambda i: rank[i]) for c, m in in_cell.items()}

        def d2(a, b):
            return int(np.sum((P[a] - P[b]) ** 2))

        for i in range(n):
            c = cell[i]
            if top[c] != i:
                assert approx[i] and dep[i] == top[c] and delta[i] == float(d_cut), i
                assert d2(i, dep[i]) < R
                continue
            # The densest point of its cell: which cells qualify?
            qual = set()
            for j in range(n):
                if cell[j] != c and d2(i, j) < R and all(rho[k] > rho[i] for k in in_cell[cell[j]]):
                    qual.add(cell[j])
            if qual:
                assert approx[i] and dep[i] == top[min(qual)] and delta[i] == float(d_cut), i
                assert rank[dep[i]] < rank[i]
            else:
                assert not approx[i] and dep[i] == ex_dep[i], i
                assert delta[i] == ex_delta[i] or (np.isinf(delta[i]) and np.isinf(ex_delta[i]))


def _impl(pts, d_cut, rho_min, delta_min):
    return approx_oracle.approx_dpc(pts, d_cut, rho_min, delta_min)


def test_cell_side():
    pin_cell_side()


def test_hand_example():
    pin_hand_example(_impl)


def test_theorem4_same_centers():
    pin_theorem4(_impl)


def test_rules_point_by_point():
    pin_rules(_impl)


def test_approximation_covers_most_points_on_blobs():
    # Not a correctness pin: the approximate rules should settle most points of a
    # clustered 2-D input, which is what makes the method pay.
    job = inputs.blob_job(33, 1500, 2, 5, 300.0, 900.0, 0.05)
    r = _impl(job.pts, job.d_cut, job.rho_min, job.delta_min)
    assert r["approx"].mean() > 0.5


# ---------------------------------------------------------------- planted mistakes

def _wrap_grid(monkeypatch, edit):
    real = approx_oracle.grid

    def fake(pts, rho, R):
        g = real(pts, rho, R)
        edit(g, np.asarray(pts, np.int64), np.asarray(rho), R)
        return g

    monkeypatch.setattr(approx_oracle, "grid", fake)


def _lowest_ranked(g, P, rho, R):
    rank = _rank(rho)
    g["pstar"] = {c: max(m, key=lambda i: rank[i]) for c, m in g["members"].items()}


def _min_rho_not_strict(g, P, rho, R):
    g["minrho"] = {c: v + 1 for c, v in g["minrho"].items()}


def _near_closed_ball(g, P, rho, R):
    for c, s in g["pstar"].items():
        d2 = np.sum((P - P[s]) ** 2, axis=1)
        g["near"][c] = sorted({g["cell"][j] for j in np.nonzero(d2 <= R)[0] if g["cell"][j] != c})


def _near_from_cell_corner(g, P, rho, R):
    # N(c) built around the first member instead of p*(c).
    for c, m in g["members"].items():
        d2 = np.sum((P - P[m[0]]) ** 2, axis=1)
        g["near"][c] = sorted({g["cell"][j] for j in np.nonzero(d2 < R)[0] if g["cell"][j] != c})


MUTANTS = {
    "lowest_ranked_pstar": _lowest_ranked,
    "min_rho_not_strict": _min_rho_not_strict,
    "near_closed_ball": _near_closed_ball,
    "near_from_first_member": _near_from_cell_corner,
}


def _some_pin_fails():
    for pin in (lambda: pin_hand_example(_impl), lambda: pin_rules(_impl), lambda: pin_theorem4(_impl)):
        try:
            pin()
        except AssertionError:
            return True
    return False


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_grid_is_caught(monkeypatch, name):
    _wrap_grid(monkeypatch, MUTANTS[name])
    assert _some_pin_fails(), name


def test_mutant_cell_side_is_caught(monkeypatch):
    real = approx_oracle.cell_side
    monkeypatch.setattr(approx_oracle, "cell_side", lambda R, d: real(R, d) + 1)
    with pytest.raises(AssertionError):
        pin_cell_side()
    # Cells one too wide also break the same-cell distance bound the rules pin
    # checks (a dense lattice has pairs at the far corners).
    assert _some_pin_fails()


def test_mutant_delta_set_to_true_distance_is_caught(monkeypatch):
    real = approx_oracle.approx_dependent

    def fake(pts, rho, d_cut):
        a = real(pts, rho, d_cut)
        P = np.asarray(pts, np.int64)
        for i in np.nonzero(a["approx"])[0]:
            a["delta"][i] = float(np.sqrt(np.sum((P[i] - P[a["dep"][i]]) ** 2)))
        return a

    monkeypatch.setattr(approx_oracle, "approx_dependent", fake)
    assert _some_pin_fails()
