"""Pins for the decision-graph oracle (Section 2.1), with no GPU: hand-worked
values, a brute force with Python's own sort, numpy's histogram2d where the bins
reduce to its convention, and planted mistakes that the pins catch."""
import math

import numpy as np
import pytest

from oracle import decision_oracle as D


def _brute_top(rho, delta, rho_min, k):
    items = sorted(((-float(delta[i]), i) for i in range(len(rho)) if rho[i] >= rho_min))
    return [i for _, i in items[:k]]


def pin_top(impl=D.top_delta):
    # hand example: ties in delta go to the smaller id; noise is left out
    rho = np.array([5, 1, 7, 5, 9, 5, 2])
    delta = np.array([3.0, 50.0, 3.0, 8.0, math.inf, 8.0, 2.0])
    ids, dl, rh = impl(rho, delta, 2, 4)
    assert ids.tolist() == [4, 3, 5, 0] and dl.tolist() == [math.inf, 8.0, 8.0, 3.0] and rh.tolist() == [9, 5, 5, 5]
    assert impl(rho, delta, 2, 100)[0].tolist() == [4, 3, 5, 0, 2, 6]
    assert impl(rho, delta, 10, 3)[0].tolist() == []
    rng = np.random.default_rng(3)
    for t in range(30):
        n = int(rng.integers(1, 300))
        rho = rng.integers(1, 8, n)
        delta = rng.integers(0, 20, n).astype(np.float64) * 0.5  # many ties
        delta[rng.integers(0, n)] = math.inf
        k = int(rng.integers(1, 40))
        got = impl(rho, delta, 3, k)[0].tolist()
        assert got == _brute_top(rho, delta, 3, k), t


def pin_histogram(impl=D.histogram):
    rho = np.array([1, 2, 2, 3, 5, 9])
    delta = np.array([0.5, 1.0, 2.0, 2.0, math.inf, 10.0])
    got = impl(rho, delta, [1, 3, 9], [0.0, 1.0, 2.0, math.inf])
    # rho bins [1,3) [3,9]; delta bins [0,1) [1,2) [2,inf]
    assert got.tolist() == [[1, 1, 1], [0, 0, 3]]
    rng = np.random.default_rng(4)
    for t in range(10):
        n = 500
        r = rng.integers(1, 50, n)
        dl = rng.uniform(0, 100, n)
        re = np.sort(rng.uniform(0, 60, 6))
        de = np.sort(rng.uniform(-5, 110, 8))
        want = np.histogram2d(r.astype(np.float64), dl, bins=[re, de])[0].astype(np.int64)
        assert np.array_equal(impl(r, dl, re, de), want), t


def pin_suggest(impl=D.suggest_delta_min):
    top = [math.inf, 900.0, 850.0, 100.0, 90.0, 80.0]
    assert impl(top, 50.0) == (850.0, 3)
    assert impl(top, 95.0) == (850.0, 3)
    assert impl(top, 900.0) == (None, 0)
    assert impl([math.inf, 400.0, 0.0], 10.0) == (400.0, 2)   # zero below: infinite ratio
    assert impl([300.0, 150.0, 75.0], 10.0) == (300.0, 1)     # equal ratios: the first pair
    assert impl([5.0], 1.0) == (None, 0)
    assert impl([], 1.0) == (None, 0)


def test_top():
    pin_top()


def test_histogram():
    pin_histogram()


def test_suggest():
    pin_suggest()


def test_mutant_ties_by_larger_id_caught():
    def bad(rho, delta, rho_min, k):
        rho = np.asarray(rho)
        ids = np.nonzero(rho >= rho_min)[0]
        order = np.lexsort((-ids, -np.asarray(delta)[ids]))
        sel = ids[order][:k]
        return sel, np.asarray(delta)[sel], rho[sel]
    with pytest.raises(AssertionError):
        pin_top(bad)


def test_mutant_open_last_bin_caught():
    with pytest.raises(AssertionError):
        pin_histogram(_open_hist)


def _open_hist(rho, delta, re, de):
    c = np.zeros((len(re) - 1, len(de) - 1), np.int64)
    for r, d in zip(rho, delta):
        i = np.searchsorted(re, r, side="right") - 1
        j = np.searchsorted(de, d, side="right") - 1
        if 0 <= i < len(re) - 1 and 0 <= j < len(de) - 1:
            c[i, j] += 1
    return c


def test_mutant_suggest_lower_side_caught():
    def bad(top, d_cut):
        dmin, _ = D.suggest_delta_min(top, d_cut)
        if dmin is None:
            return None, 0
        j = list(top).index(dmin)
        lo = top[j + 1]
        return lo, sum(1 for x in top if x >= lo)
    with pytest.raises(AssertionError):
        pin_suggest(bad)
