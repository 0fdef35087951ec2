"""Pins for the oracle: checks that tie it to something other than itself.

Each ``pin_*`` function takes an oracle implementation (a module-like object
with ``local_density``, ``dependent``, ``dependent_distance``, ``labels``) and
raises AssertionError when the implementation disagrees with:

* the hand-worked example (tests/golden/hand_example.json, Defs. 1-6);
* a pure-Python brute force written straight from Defs. 1-6, deciding
  ``dist < d_cut`` with exact rationals instead of an integer threshold, and
  labelling by walking dependency chains instead of a depth-first search;
* scipy's kd-tree (ball counts and pair counts);
* a 1-D version of the paper's incremental idea (Section 3, dependent point
  computation): insert points in density order into a sorted structure and
  answer each nearest-neighbour query among the points already inserted;
* closed-form special cases and metamorphic relations.

The test modules run every pin on the real oracle, and run them on oracles
with planted mistakes to show that each mistake is caught.
"""
from __future__ import annotations

import bisect
import json
import math
import os
from fractions import Fraction

import numpy as np

from paper_2207_04649_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_example.json")
INF_D2 = np.iinfo(np.int64).max


# ---------------------------------------------------------------- helpers

def brute_dpc(pts, d_cut, rho_min, delta_min):
    """Defs. 1-6 by plain loops; no sorting, no integer cut-off."""
    P = [tuple(int(v) for v in row) for row in np.asarray(pts)]
    n = len(P)
    dc2 = Fraction(d_cut) ** 2

    def d2(a, b):
        return sum((x - y) ** 2 for x, y in zip(a, b))

    rho = [sum(1 for j in range(n) if Fraction(d2(P[i], P[j])) < dc2) for i in range(n)]

    def higher(j, i):  # j ranks above i
        return rho[j] > rho[i] or (rho[j] == rho[i] and j < i)

    dep, dd = [], []
    for i in range(n):
        best = None
        for j in range(n):
            if j != i and higher(j, i):
                key = (d2(P[i], P[j]), j)
                if best is None or key < best:
                    best = key
        dep.append(-1 if best is None else best[1])
        dd.append(INF_D2 if best is None else best[0])
    delta = [math.inf if x == INF_D2 else math.sqrt(x) for x in dd]
    noise = [r < rho_min for r in rho]
    center = [not noise[i] and delta[i] >= delta_min for i in range(n)]
    label = []
    for i in range(n):
        if noise[i]:
            label.append(-1)
            continue
        u = i
        while not center[u]:
            u = dep[u]
        label.append(u)
    return {"rho": rho, "dep": dep, "d2": dd, "delta": delta, "label": label,
            "ncenters": sum(center)}


def run(impl, pts, d_cut, rho_min, delta_min):
    rho = np.asarray(impl.local_density(pts, d_cut))
    dep, d2 = impl.dependent(pts, rho)
    delta = np.asarray(impl.dependent_distance(d2))
    lab, nc = impl.labels(rho, dep, delta, rho_min, delta_min)
    return {"rho": rho, "dep": np.asarray(dep), "d2": np.asarray(d2), "delta": delta,
            "label": np.asarray(lab), "ncenters": nc}


def assert_same(got, want, keys=("rho", "dep", "d2", "delta", "label", "ncenters"), ctx=""):
    for k in keys:
        a, b = got[k], want[k]
        if k == "delta":
            assert np.array_equal(np.asarray(a, np.float64).view(np.int64),
                                  np.asarray(b, np.float64).view(np.int64)), f"{ctx} {k}"
        else:
            assert np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64)), f"{ctx} {k}: {a} vs {b}"


def rank_of(rho):
    rho = np.asarray(rho, np.int64)
    order = sorted(range(rho.size), key=lambda i: (-int(rho[i]), i))
    rank = np.empty(rho.size, np.int64)
    rank[order] = np.arange(rho.size)
    return rank


# ---------------------------------------------------------------- pins

def pin_hand_example(impl):
    g = json.load(open(GOLDEN))
    P = np.array(g["points"], np.int32)
    for case in g["cases"]:
        rho = np.asarray(impl.local_density(P, case["d_cut"]))
        assert rho.tolist() == case["rho"], ("rho", case["d_cut"])
        dep, d2 = impl.dependent(P, rho)
        assert np.asarray(dep).tolist() == case["dep"], ("dep", case["d_cut"])
        if "d2" in case:
            want = [INF_D2 if v is None else v for v in case["d2"]]
            assert np.asarray(d2).tolist() == want, ("d2", case["d_cut"])
        delta = np.asarray(impl.dependent_distance(d2))
        if "delta" in case:
            assert delta.tolist() == case["delta"], ("delta", case["d_cut"])
        for lc in case["labels"]:
            lab, nc = impl.labels(rho, dep, delta, lc["rho_min"], lc["delta_min"])
            assert np.asarray(lab).tolist() == lc["label"], ("label", case["d_cut"], lc)
            assert nc == len(lc["centers"])


def brute_cases():
    """Tiny inputs: small domains force duplicate points and distance ties."""
    cases = []
    for seed in range(6):
        for d in (1, 2, 3, 5, 8):
            for n in (1, 2, 9, 60):
                hi = [3, 12, 40][seed % 3]
                d_cut = [1.0, 2.5, 4.0, 7.3][(seed + d) % 4]
                cases.append((inputs.uniform_points(n, d, hi, 1000 * seed + 10 * d + n), d_cut,
                              1 + seed % 3, d_cut * 1.5))
    lat = inputs.lattice_points(5, 2, 3)
    cases.append((lat, 3.0, 2, 4.0))   # D2 = 9 = R exactly on every axis pair
    cases.append((lat, 3.01, 2, 4.0))
    return cases


def pin_brute_force(impl, cases=None):
    for pts, d_cut, rho_min, delta_min in (cases or brute_cases()):
        assert_same(run(impl, pts, d_cut, rho_min, delta_min),
                    brute_dpc(pts, d_cut, rho_min, delta_min), ctx=f"n={len(pts)} d_cut={d_cut}")


def pin_scipy_density(impl):
    """rho against kd-tree ball counts at radius sqrt(R - 1/2); sum(rho) against
    n + 2 * (kd-tree pair count).  R is derived here from rationals."""
    from scipy.spatial import cKDTree

    for seed, (n, d, d_cut) in enumerate([(1500, 2, 700.0), (1200, 3, 1500.5), (800, 5, 2200.0), (600, 1, 150.25)]):
        job = inputs.blob_job(seed + 77, n, d, 4, 500.0, 1500.0, 0.1)
        pts = job.pts
        R = math.ceil(Fraction(d_cut) ** 2)
        tree = cKDTree(pts.astype(np.float64))
        r = math.sqrt(R - 0.5)
        want = tree.query_ball_point(pts.astype(np.float64), r=r, return_length=True)
        rho = np.asarray(impl.local_density(pts, d_cut))
        assert np.array_equal(rho, want), ("rho vs kd-tree", n, d)
        pairs = len(tree.query_pairs(r=r))
        assert int(rho.sum()) == n + 2 * pairs, "sum(rho) = n + 2 * pairs"


def pin_dependent_certificate(impl):
    """For every point, the kd-tree ball of radius sqrt(D2_i + 1/2) holds every
    point at squared distance <= D2_i; the (D2, id)-smallest higher-ranked one
    among them must be dep_i, and no higher point may be strictly closer.  The
    ranks use kd-tree densities, not the implementation's."""
    from scipy.spatial import cKDTree

    for seed, (n, d, d_cut) in enumerate([(1200, 2, 500.0), (700, 4, 2500.0)]):
        job = inputs.blob_job(seed + 300, n, d, 5, 400.0, 1200.0, 0.15)
        pts = job.pts.astype(np.int64)
        fp = pts.astype(np.float64)
        tree = cKDTree(fp)
        R = math.ceil(Fraction(d_cut) ** 2)
        rho_t = tree.query_ball_point(fp, r=math.sqrt(R - 0.5), return_length=True)
        rank = rank_of(rho_t)
        dep, d2 = impl.dependent(job.pts, np.asarray(impl.local_density(job.pts, d_cut)))
        dep = np.asarray(dep)
        d2 = np.asarray(d2)
        top = int(np.argmin(rank))
        for i in range(n):
            if i == top:
                assert dep[i] == -1 and d2[i] == INF_D2
                continue
            ball = tree.query_ball_point(fp[i], r=math.sqrt(float(d2[i]) + 0.5))
            ball = np.array([j for j in ball if rank[j] < rank[i]], np.int64)
            assert ball.size, ("no higher point within D2", i)
            dd = np.sum((pts[ball] - pts[i]) ** 2, axis=1)
            best = min(zip(dd.tolist(), ball.tolist()))
            assert best == (int(d2[i]), int(dep[i])), ("dependent", i, best, d2[i], dep[i])


def incremental_1d(x, rho):
    """Dependent points in 1-D the way Ex-DPC builds them (Section 3): visit
    points in density order and query the nearest among those inserted so far,
    using a sorted list instead of a kd-tree.  Ties: smaller id."""
    n = len(x)
    order = sorted(range(n), key=lambda i: (-int(rho[i]), i))
    keys: list[tuple[int, int]] = []  # (coordinate, id), sorted
    dep = [-1] * n
    d2 = [INF_D2] * n
    for i in order:
        xi = int(x[i])
        if keys:
            cands = []
            k = bisect.bisect_left(keys, (xi, -1))
            if k < len(keys):                      # nearest at or right of xi
                cands.append(keys[k])
            if k > 0:                              # nearest left of xi: smallest id there
                xl = keys[k - 1][0]
                cands.append(keys[bisect.bisect_left(keys, (xl, -1))])
            best = min(((c[0] - xi) ** 2, c[1]) for c in cands)
            d2[i], dep[i] = best
        bisect.insort(keys, (xi, i))
    return dep, d2


def pin_incremental_1d(impl):
    for seed, (n, hi, d_cut) in enumerate([(400, 300, 6.0), (1500, 100_000, 900.0), (300, 20, 1.5)]):
        pts = inputs.uniform_points(n, 1, hi, 5000 + seed)
        from scipy.spatial import cKDTree
        fp = pts.astype(np.float64)
        R = math.ceil(Fraction(d_cut) ** 2)
        rho_t = cKDTree(fp).query_ball_point(fp, r=math.sqrt(R - 0.5), return_length=True)
        want_dep, want_d2 = incremental_1d(pts[:, 0], rho_t)
        rho = np.asarray(impl.local_density(pts, d_cut))
        dep, d2 = impl.dependent(pts, rho)
        assert np.asarray(dep).tolist() == want_dep
        assert np.asarray(d2).tolist() == want_d2


def pin_special_cases(impl):
    # S1: d_cut beyond every distance -> rho = n, rank = id order, dep = nearest earlier id.
    pts = inputs.uniform_points(120, 3, 50, 11)
    rho = np.asarray(impl.local_density(pts, 1000.0))
    assert (rho == 120).all()
    dep, d2 = impl.dependent(pts, rho)
    p = pts.astype(np.int64)
    for i in range(1, 120):
        dd = np.sum((p[:i] - p[i]) ** 2, axis=1)
        j = int(np.argmin(dd))  # argmin returns the first, i.e. smallest id
        assert (int(dep[i]), int(d2[i])) == (j, int(dd[j]))
    assert dep[0] == -1
    # S2: R = 1 -> rho is the coordinate multiplicity.
    pts = inputs.uniform_points(300, 2, 6, 12)
    rho = np.asarray(impl.local_density(pts, 0.75))
    _, inv, cnt = np.unique(pts, axis=0, return_inverse=True, return_counts=True)
    assert np.array_equal(rho, cnt[inv.ravel()])
    # S3: a single point.
    one = np.array([[5, 7, 9]], np.int32)
    rho = np.asarray(impl.local_density(one, 10.0))
    dep, d2 = impl.dependent(one, rho)
    delta = np.asarray(impl.dependent_distance(d2))
    lab, nc = impl.labels(rho, dep, delta, 1, 20.0)
    assert rho.tolist() == [1] and np.asarray(dep).tolist() == [-1]
    assert math.isinf(delta[0]) and np.asarray(lab).tolist() == [0] and nc == 1
    lab, nc = impl.labels(rho, dep, delta, 2, 20.0)
    assert np.asarray(lab).tolist() == [-1] and nc == 0


def pin_invariants(impl):
    job = inputs.blob_job(901, 2500, 2, 6, 600.0, 1500.0, 0.08)
    out = run(impl, job.pts, job.d_cut, job.rho_min, job.delta_min)
    rho, dep, d2, delta, lab = out["rho"], out["dep"], out["d2"], out["delta"], out["label"]
    rank = rank_of(rho)
    tops = np.nonzero(dep < 0)[0]
    assert tops.tolist() == [int(np.argmin(rank))], "exactly one point without a dependent"
    rest = dep >= 0
    assert (rank[dep[rest]] < rank[rest]).all(), "dependent ranks higher (I2)"
    p = job.pts.astype(np.int64)
    idx = np.nonzero(rest)[0]
    exact = np.sum((p[idx] - p[dep[idx]]) ** 2, axis=1)
    assert np.array_equal(exact, d2[idx]), "d2 is the distance to dep"
    assert np.array_equal(np.sqrt(exact.astype(np.float64)), delta[idx]), "delta = sqrt(D2) (I3)"
    noise = rho < job.rho_min
    center = ~noise & (delta >= job.delta_min)
    assert ((lab == -1) == noise).all(), "I5 noise"
    assert (lab[center] == np.nonzero(center)[0]).all(), "I5 centers"
    other = ~noise & ~center
    assert (lab[other] == lab[dep[other]]).all(), "I5 propagation"
    assert out["ncenters"] == int(center.sum()), "I6"
    # I7: labels are a function of (rho, dep, delta, thresholds) only.
    for rm, dm in [(1, job.delta_min), (30, 2 * job.delta_min), (5, job.d_cut * 1.01)]:
        lab2, _ = impl.labels(rho, dep, delta, rm, dm)
        want = brute_labels(rho, dep, delta, rm, dm)
        assert np.array_equal(np.asarray(lab2), want)


def brute_labels(rho, dep, delta, rho_min, delta_min):
    n = len(rho)
    out = np.full(n, -1, np.int64)
    for i in range(n):
        if rho[i] < rho_min:
            continue
        u = i
        while not (delta[u] >= delta_min):
            u = int(dep[u])
        out[i] = u
    return out


def pin_metamorphic(impl):
    job = inputs.blob_job(902, 900, 3, 4, 500.0, 1200.0, 0.1)
    base = run(impl, job.pts, job.d_cut, job.rho_min, job.delta_min)
    shifted = job.pts.astype(np.int64) + np.array([17, -3, 5])
    shifted -= shifted.min(axis=0)
    assert_same(run(impl, shifted.astype(np.int32), job.d_cut, job.rho_min, job.delta_min), base, ctx="translate")
    perm = np.ascontiguousarray(job.pts[:, [2, 0, 1]])
    assert_same(run(impl, perm, job.d_cut, job.rho_min, job.delta_min), base, ctx="permute")
    big = run(impl, job.pts * 2, 2 * job.d_cut, job.rho_min, 2 * job.delta_min)
    assert_same(big, base, keys=("rho", "dep", "label", "ncenters"), ctx="scale")
    ok = base["dep"] >= 0
    assert np.array_equal(big["d2"][ok], 4 * base["d2"][ok])
    assert np.array_equal(big["delta"], 2 * base["delta"])


ALL_PINS = [pin_hand_example, pin_brute_force, pin_scipy_density, pin_dependent_certificate,
            pin_incremental_1d, pin_special_cases, pin_invariants, pin_metamorphic]
