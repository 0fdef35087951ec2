"""Plant plausible mistakes in a copy of the numpy oracle and check that the
pins catch each one (no GPU).  A pin set that let one of these through would
not be pinning the oracle."""
import math
import types

import numpy as np
import pytest

from oracle import dpc_oracle as base
from tests import oracle_pins as pins


def _mutant(**overrides):
    m = types.SimpleNamespace(local_density=base.local_density, dependent=base.dependent,
                              dependent_distance=base.dependent_distance, labels=base.labels)
    for k, v in overrides.items():
        setattr(m, k, v)
    return m


def _rho_with(cmp, self_count=True):
    def f(pts, d_cut):
        p = np.asarray(pts, np.int64)
        R = base.cutoff_square(d_cut)
        D2 = np.sum((p[:, None, :] - p[None, :, :]) ** 2, axis=2)
        inside = cmp(D2, R)
        if not self_count:
            np.fill_diagonal(inside, False)
        return np.count_nonzero(inside, axis=1)
    return f


def _rho_floor(pts, d_cut):  # R = floor(d_cut^2) instead of ceil
    p = np.asarray(pts, np.int64)
    R = math.floor(d_cut * d_cut)
    D2 = np.sum((p[:, None, :] - p[None, :, :]) ** 2, axis=2)
    return np.count_nonzero(D2 < R, axis=1)


def _dep_with(order_key, tie_larger_id=False, transposed=False):
    def f(pts, rho):
        p = np.asarray(pts, np.int64)
        rho = np.asarray(rho, np.int64)
        n = p.shape[0]
        order = np.array(sorted(range(n), key=lambda i: order_key(rho, i)), np.int64)
        rank = np.empty(n, np.int64)
        rank[order] = np.arange(n)
        dep = np.full(n, -1, np.int64)
        d2 = np.full(n, pins.INF_D2, np.int64)
        for i in range(n):
            r = rank[i]
            if r == 0:
                continue
            cand = order[:r]
            q = p[cand[0]] if transposed else p[i]
            dd = np.sum((p[cand] - q) ** 2, axis=1) if not transposed else np.sum((p[cand] - p[i][::-1]) ** 2, axis=1)
            best = dd.min()
            ids = cand[dd == best]
            dep[i] = ids.max() if tie_larger_id else ids.min()
            d2[i] = best
        return dep, d2
    return f


def _delta_f32(d2):
    out = np.sqrt(np.asarray(d2).astype(np.float32)).astype(np.float64)
    out[np.asarray(d2) == pins.INF_D2] = np.inf
    return out


def _labels_strict(rho, dep, delta, rho_min, delta_min):
    return base.labels(rho, dep, np.where(np.asarray(delta) == delta_min, -1.0, delta), rho_min, delta_min)


def _labels_noise_joins(rho, dep, delta, rho_min, delta_min):
    lab, nc = base.labels(rho, dep, delta, rho_min - 1, delta_min)
    return lab, nc


MUTANTS = {
    "rho_le": _mutant(local_density=_rho_with(lambda D2, R: D2 <= R)),
    "rho_no_self": _mutant(local_density=_rho_with(lambda D2, R: D2 < R, self_count=False)),
    "rho_floor_cutoff": _mutant(local_density=_rho_floor),
    "dep_tie_larger_id": _mutant(dependent=_dep_with(lambda r, i: (-r[i], i), tie_larger_id=True)),
    "rank_tie_larger_id": _mutant(dependent=_dep_with(lambda r, i: (-r[i], -i))),
    "rank_ascending": _mutant(dependent=_dep_with(lambda r, i: (r[i], i))),
    "dep_transposed_operand": _mutant(dependent=_dep_with(lambda r, i: (-r[i], i), transposed=True)),
    "delta_f32": _mutant(dependent_distance=_delta_f32),
    "center_strict": _mutant(labels=_labels_strict),
    "noise_off_by_one": _mutant(labels=_labels_noise_joins),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_catch(name):
    mutant = MUTANTS[name]
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin caught the planted mistake {name}"
