"""Pins for the S-Approx-DPC oracle (Section 5), with no GPU.

* Cells of side 1 (eps * d_cut <= 1): every distinct point is its cell's pick,
  duplicates share a cell whose pick is their smallest id, and the result must
  equal the exact method's oracle in every output: the first phase then takes
  the nearest higher-ranked point within d_cut, which is the exact dependent point
  whenever that lies within d_cut, and the second phase is the exact search.
* Bounds the section states: a point that was not picked lies within eps * d_cut
  of its pick, a first-phase dependent point within (1 + eps) d_cut.
* The picks' densities are exact (Def. 1) and the second phase returns the
  exact nearest higher-ranked pick (the exact oracle run on the picks alone).
* Planted mistakes are caught.
"""
import math

import numpy as np
import pytest

from oracle import dpc_oracle, sapprox_oracle as S
from paper_2207_04649_amd import inputs


def _cases():
    out = []
    for seed in range(3):
        for d in (1, 2, 3, 4):
            hi = [30, 200, 3000][seed]
            d_cut = [2.5, 6.0, 40.0, 300.0][(seed + d) % 4]
            out.append((inputs.uniform_points(150, d, hi, 700 + 10 * seed + d), d_cut))
    job = inputs.blob_job(51, 500, 2, 4, 300.0, 900.0, 0.1)
    out.append((job.pts, job.d_cut))
    out.append((inputs.lattice_points(10, 2, 1), 3.0))
    return out


def pin_unit_cells_equal_exact(impl):
    for pts, d_cut in _cases():
        eps = 0.9 / d_cut  # eps * d_cut < 1: cells of side 1
        r = impl(pts, d_cut, eps, 2, 1.5 * d_cut)
        ex = dpc_oracle.dpc(pts, d_cut, 2, 1.5 * d_cut)
        for k in ("rho", "dep", "label"):
            assert np.array_equal(r[k], ex[k]), (k, d_cut)
        assert np.array_equal(r["delta"].view(np.int64), ex["delta"].view(np.int64))


def pin_bounds_and_phases(impl):
    for pts, d_cut in _cases():
        P = np.asarray(pts, np.int64)
        for eps in (0.3, 0.7, 1.0):
            r = impl(P, d_cut, eps, 2, 1.5 * d_cut)
            side = r["side"]
            assert d_cut * eps >= 1.0 or side == 1
            assert P.shape[1] * (side - 1) ** 2 < (eps * d_cut) ** 2 or side == 1
            picked = r["picked"]
            pick_ids = np.nonzero(picked)[0]
            rho_exact = dpc_oracle.local_density(P, d_cut)
            assert np.array_equal(r["rho"][picked], rho_exact[picked])
            # the second phase equals the exact search over the picks alone
            sub_dep, sub_d2 = dpc_oracle.dependent(P[pick_ids], r["rho"][pick_ids])
            for i in range(P.shape[0]):
                if not picked[i]:
                    q = r["dep"][i]
                    assert picked[q] and q < i and r["rho"][i] == r["rho"][q]
                    assert tuple(P[i] // side) == tuple(P[q] // side)
                    assert r["delta"][i] < eps * d_cut
                elif r["phase"][i] == 1:
                    assert picked[r["dep"][i]]
                    assert r["delta"][i] < (1 + eps) * d_cut
            for k, i in enumerate(pick_ids):
                if r["phase"][i] == 2:
                    want = -1 if sub_dep[k] < 0 else pick_ids[sub_dep[k]]
                    assert r["dep"][i] == want, i


def _impl(pts, d_cut, eps, rho_min, delta_min):
    return S.sapprox_dpc(pts, d_cut, eps, rho_min, delta_min)


def test_unit_cells_equal_exact():
    pin_unit_cells_equal_exact(_impl)


def test_bounds_and_phases():
    pin_bounds_and_phases(_impl)


def test_eps_range():
    for bad in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(ValueError):
            S.sapprox_dpc(np.zeros((3, 2), np.int32), 5.0, bad, 1, 6.0)


def test_fewer_picks_as_eps_grows():
    job = inputs.blob_job(52, 1500, 2, 5, 300.0, 900.0, 0.05)
    counts = [int(S.sapprox_dpc(job.pts, job.d_cut, e, job.rho_min, job.delta_min)["picked"].sum())
              for e in (0.2, 0.5, 1.0)]
    assert counts[0] > counts[1] > counts[2]


# ---------------------------------------------------------------- planted mistakes

def _all_pins():
    for pin in (pin_unit_cells_equal_exact, pin_bounds_and_phases):
        try:
            pin(_impl)
        except AssertionError:
            return True
    return False


MUTANTS = {
    "pick_largest_id": ("pick_of", lambda real: (lambda ids: max(ids))),
    "side_too_wide": ("cell_side", lambda real: (lambda Re, d: real(Re, d) + 1)),
    "closed_ball": ("within", lambda real: (lambda d2, R: d2 <= R)),
    "farthest_candidate": ("nearest", lambda real: (lambda p, i, c: max((int(np.sum((p[i] - p[q]) ** 2)), int(q))
                                                                        for q in c))),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_caught(monkeypatch, name):
    attr, make = MUTANTS[name]
    monkeypatch.setattr(S, attr, make(getattr(S, attr)))
    assert _all_pins(), name


def _rand_index(a, b):
    """Rand index of two labelings (noise, -1, counts as one more cluster)."""
    _, ia = np.unique(np.asarray(a), return_inverse=True)
    _, ib = np.unique(np.asarray(b), return_inverse=True)
    m = np.zeros((ia.max() + 1, ib.max() + 1), np.int64)
    np.add.at(m, (ia.reshape(-1), ib.reshape(-1)), 1)
    c2 = lambda x: int((x * (x - 1) // 2).sum())  # noqa: E731
    n = ia.size
    tot = n * (n - 1) // 2
    return (tot + 2 * c2(m) - c2(m.sum(1)) - c2(m.sum(0))) / tot


def test_rand_index_falls_as_eps_grows():
    # The trend of Table 5 (weak: the section claims no guarantee), on two seeded
    # blob jobs: the Rand index against the exact labels does not rise with eps,
    # and fewer points are picked.  Approx-DPC keeps the exact clustering here.
    from oracle import approx_oracle
    for seed in (61, 62):
        job = inputs.blob_job(seed, 3000, 2, 6, 500.0, 2500.0, 0.05)
        ex = dpc_oracle.dpc(job.pts, job.d_cut, job.rho_min, job.delta_min)
        ax = approx_oracle.approx_dpc(job.pts, job.d_cut, job.rho_min, job.delta_min)
        assert _rand_index(ex["label"], ax["label"]) >= 0.999
        ri, picks = [], []
        for eps in (0.1, 0.4, 0.7, 1.0):
            sx = S.sapprox_dpc(job.pts, job.d_cut, eps, job.rho_min, job.delta_min)
            ri.append(_rand_index(ex["label"], sx["label"]))
            picks.append(int(sx["picked"].sum()))
        assert all(a >= b for a, b in zip(ri, ri[1:])), ri
        assert all(a > b for a, b in zip(picks, picks[1:])), picks
        assert ri[-1] > 0.95
