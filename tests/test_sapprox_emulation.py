"""S-Approx-DPC's kernel sources run on the CPU (tests/cpu_emu) against the
S-Approx-DPC oracle, element by element: rho, dep, delta (bit for bit), the
picked flags, labels and the number of centers."""
import os

import numpy as np
import pytest

from oracle import sapprox_oracle
from paper_2207_04649_amd import inputs
from tests.cpu_emu import build_emu
from tests.test_cpu_emulation import _parse, _record, _run

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe():
    return build_emu.build(os.path.join(ROOT, "_build", "emu"), asan=True)


def run_sapprox_emu(exe, pts, d_cut, eps, rho_min, delta_min):
    n = int(np.asarray(pts).shape[0])
    b = _run(exe, ["--sapprox", repr(float(eps))], _record(pts, d_cut, rho_min, delta_min))
    out, o = _parse(b, 0, n)
    out["picked"] = np.frombuffer(b, np.uint8, n, o).copy()
    return out


def check(got, pts, d_cut, eps, rho_min, delta_min, ctx=""):
    want = sapprox_oracle.sapprox_dpc(pts, d_cut, eps, rho_min, delta_min)
    assert got["status"] == 0 and got["sync"] == 0, ctx
    assert np.array_equal(got["picked"].astype(bool), want["picked"]), ctx
    assert np.array_equal(got["rho"], want["rho"]), ctx
    assert np.array_equal(got["dep"], want["dep"]), ctx
    assert np.array_equal(got["delta"].view(np.int64), want["delta"].view(np.int64)), ctx
    assert np.array_equal(got["label"], want["label"]), ctx
    assert got["ncenters"] == want["ncenters"], ctx


# (eps 0.3 on the first seed, 1.0 on the second: the suite stays within minutes)
CASES = [(seed, d, n, dc, (0.3, 1.0)[seed]) for seed in range(2)
         for d, dc, ns in [(1, 40.0, (3, 700)), (2, 300.0, (1, 200, 700)), (2, 3000.0, (200,)),
                           (3, 2000.0, (200,)), (4, 4500.0, (150,)), (6, 14000.0, (40,)), (8, 27000.0, (12,))]
         for n in ns]


@pytest.mark.parametrize("seed,d,n,d_cut,eps", CASES)
def test_emulated_sapprox_matches_oracle(emu_exe, seed, d, n, d_cut, eps):
    hi = [20000, 131071][seed]
    pts = inputs.uniform_points(n, d, hi, 1300 + 31 * seed + d * 7 + n)
    check(run_sapprox_emu(emu_exe, pts, d_cut, eps, 2, 1.5 * d_cut), pts, d_cut, eps, 2, 1.5 * d_cut,
          (seed, d, n, eps))


def test_emulated_sapprox_blobs(emu_exe):
    job = inputs.blob_job(43, 1200, 2, 5, 600.0, 2000.0, 0.1)
    eps = 0.4
    check(run_sapprox_emu(emu_exe, job.pts, job.d_cut, eps, job.rho_min, job.delta_min), job.pts, job.d_cut,
          eps, job.rho_min, job.delta_min, eps)


def test_emulated_sapprox_edges(emu_exe):
    dup = np.repeat(inputs.uniform_points(30, 2, 4, 5), 4, axis=0) * 50
    check(run_sapprox_emu(emu_exe, dup, 120.0, 0.5, 1, 200.0), dup, 120.0, 0.5, 1, 200.0, "dup")
    lat = inputs.lattice_points(15, 2, 100)
    check(run_sapprox_emu(emu_exe, lat, 300.0, 1.0, 2, 400.0), lat, 300.0, 1.0, 2, 400.0, "lattice")
    one = np.zeros((1, 3), np.int32)
    check(run_sapprox_emu(emu_exe, one, 50.0, 0.5, 1, 60.0), one, 50.0, 0.5, 1, 60.0, "single")
    # unit cells: equals the exact method
    pts = inputs.uniform_points(300, 2, 25, 17) * 40
    check(run_sapprox_emu(emu_exe, pts, 90.0, 0.01, 1, 100.0), pts, 90.0, 0.01, 1, 100.0, "unit cells")
    # every point within d_cut of every other: some picks have density n
    close = inputs.uniform_points(40, 3, 30, 21)
    check(run_sapprox_emu(emu_exe, close, 200.0, 0.1, 1, 300.0), close, 200.0, 0.1, 1, 300.0, "dense")
