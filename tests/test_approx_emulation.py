"""Approx-DPC's kernel sources run on the CPU (tests/cpu_emu) against the
Approx-DPC oracle, element by element: rho, dep, delta (bit for bit), the
approx flags, labels and the number of centers."""
import os

import numpy as np
import pytest

from oracle import approx_oracle
from paper_2207_04649_amd import inputs
from tests.cpu_emu import build_emu
from tests.test_cpu_emulation import _parse, _record, _run

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe():
    return build_emu.build(os.path.join(ROOT, "_build", "emu"), asan=True)


def run_approx_emu(exe, pts, d_cut, rho_min, delta_min):
    n = int(np.asarray(pts).shape[0])
    b = _run(exe, ["--approx"], _record(pts, d_cut, rho_min, delta_min))
    out, o = _parse(b, 0, n)
    out["approx"] = np.frombuffer(b, np.uint8, n, o).copy()
    return out


def check(got, pts, d_cut, rho_min, delta_min, ctx=""):
    want = approx_oracle.approx_dpc(pts, d_cut, rho_min, delta_min)
    assert got["status"] == 0 and got["sync"] == 0, ctx
    assert np.array_equal(got["rho"], want["rho"]), ctx
    assert np.array_equal(got["approx"].astype(bool), want["approx"]), ctx
    assert np.array_equal(got["dep"], want["dep"]), ctx
    assert np.array_equal(got["delta"].view(np.int64), want["delta"].view(np.int64)), ctx
    assert np.array_equal(got["label"], want["label"]), ctx
    assert got["ncenters"] == want["ncenters"], ctx


# Cut-offs keep the exact grid's dense cell table small enough to emulate.
# (the larger sizes on the first seed only: the suite stays within minutes)
CASES = [(seed, d, n, dc) for seed in range(2)
         for d, dc, ns in [(1, 40.0, (3, 700)), (2, 300.0, (1, 200, 700)), (2, 3000.0, (200,)),
                           (3, 2000.0, (200,)), (4, 4500.0, (150,)), (6, 14000.0, (40,)), (8, 27000.0, (12,))]
         for n in ns if seed == 0 or n < 500]


@pytest.mark.parametrize("seed,d,n,d_cut", CASES)
def test_emulated_approx_matches_oracle(emu_exe, seed, d, n, d_cut):
    hi = [20000, 131071][seed]
    pts = inputs.uniform_points(n, d, hi, 900 + 31 * seed + d * 7 + n)
    check(run_approx_emu(emu_exe, pts, d_cut, 2, 1.5 * d_cut), pts, d_cut, 2, 1.5 * d_cut, (seed, d, n))


def test_emulated_approx_blobs(emu_exe):
    job = inputs.blob_job(41, 1200, 2, 5, 600.0, 2000.0, 0.1)
    check(run_approx_emu(emu_exe, job.pts, job.d_cut, job.rho_min, job.delta_min), job.pts, job.d_cut,
          job.rho_min, job.delta_min)


def test_emulated_approx_duplicates_and_lattice(emu_exe):
    # many equal points (one cell, equal densities) and a lattice at D2 = R exactly
    dup = np.repeat(inputs.uniform_points(30, 2, 4, 5), 4, axis=0) * 50
    check(run_approx_emu(emu_exe, dup, 120.0, 1, 200.0), dup, 120.0, 1, 200.0, "dup")
    lat = inputs.lattice_points(15, 2, 100)
    check(run_approx_emu(emu_exe, lat, 300.0, 2, 400.0), lat, 300.0, 2, 400.0, "lattice")
    one = np.zeros((1, 3), np.int32)
    check(run_approx_emu(emu_exe, one, 50.0, 1, 60.0), one, 50.0, 1, 60.0, "single")


def test_emulated_approx_tiny_cut(emu_exe):
    # d_cut <= 1: cells of side 1, only duplicates share a cell
    pts = inputs.uniform_points(300, 2, 25, 17) * 40
    check(run_approx_emu(emu_exe, pts, 0.9, 1, 1.0), pts, 0.9, 1, 1.0, "tiny")
