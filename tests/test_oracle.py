"""The oracle against its pins (no GPU): both the numpy and the C oracle."""
import numpy as np
import pytest

from oracle import dpc_oracle, scan
from paper_2207_04649_amd import inputs
from tests import oracle_pins as pins

IMPLS = {"numpy": dpc_oracle, "c": scan}


@pytest.mark.parametrize("impl", list(IMPLS))
@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(impl, pin):
    pin(IMPLS[impl])


def test_cutoff_square_closed_forms():
    R = dpc_oracle.cutoff_square
    assert R(3.0) == 9
    assert R(2.8) == 8          # 2.8**2 = 7.84 (binary value slightly below)
    assert R(0.5) == 1 and R(1.0) == 1 and R(1e-300) == 1
    assert R(2.0 ** 20) == 2 ** 40
    assert R(1000.0) == 1_000_000
    # The double nearest sqrt(2) lies above sqrt(2): its exact square exceeds 2,
    # so a pair at D2 = 2 is strictly inside.
    import math
    assert R(math.sqrt(2.0)) == 3
    assert R(math.nextafter(3.0, 0.0)) == 9 and R(math.nextafter(3.0, 4.0)) == 10
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            R(bad)


def test_c_matches_numpy_random():
    for seed in range(4):
        for d in (1, 2, 4, 7):
            pts = inputs.uniform_points(700, d, [50, 400, 5000, 100000][seed], seed * 10 + d)
            d_cut = [3.0, 40.5, 900.0, 20000.0][seed]
            a = pins.run(dpc_oracle, pts, d_cut, 3, 2 * d_cut)
            b = pins.run(scan, pts, d_cut, 3, 2 * d_cut)
            pins.assert_same(b, a, ctx=f"seed={seed} d={d}")


def test_c_dependent_of_matches_full():
    job = inputs.blob_job(77, 3000, 2, 5, 500.0, 1500.0, 0.1)
    full = pins.run(scan, job.pts, job.d_cut, job.rho_min, job.delta_min)
    which = np.arange(0, 3000, 7)
    rho, dep, d2 = scan.dependent_of(job.pts, job.d_cut, which)
    assert np.array_equal(rho, full["rho"][which])
    assert np.array_equal(dep, full["dep"][which])
    assert np.array_equal(d2, full["d2"][which])
    assert np.array_equal(scan.local_density_of(job.pts, job.d_cut, which), full["rho"][which])
    # A walk limit marks undecided points and leaves the others exact.
    rho, dep, d2 = scan.dependent_of(job.pts, job.d_cut, which, max_walk=3)
    ok = dep != -2
    assert ok.any() and (~ok).any()
    assert np.array_equal(dep[ok], full["dep"][which][ok])


def test_c_matches_numpy_blobs_20k():
    job = inputs.blobs_20k()
    a = pins.run(dpc_oracle, job.pts, job.d_cut, job.rho_min, job.delta_min)
    b = pins.run(scan, job.pts, job.d_cut, job.rho_min, job.delta_min)
    pins.assert_same(b, a, ctx="blobs_20k")
