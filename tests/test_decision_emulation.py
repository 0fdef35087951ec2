"""The decision-graph kernels run on the CPU (tests/cpu_emu) against the
decision-graph oracle: top-k ids, deltas and rhos bit for bit, the suggested
delta_min and its count of centers, and the <rho, delta> histogram counts."""
import math
import os
import struct

import numpy as np
import pytest

from oracle import approx_oracle, decision_oracle as D, dpc_oracle
from paper_2207_04649_amd import inputs
from tests.cpu_emu import build_emu
from tests.test_cpu_emulation import _run

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe():
    return build_emu.build(os.path.join(ROOT, "_build", "emu"), asan=True)


def run_decision_emu(exe, rho, delta, rho_min, k, d_cut, re, de):
    rho = np.ascontiguousarray(rho, np.int32)
    delta = np.ascontiguousarray(delta, np.float64)
    re = np.ascontiguousarray(re, np.float64)
    de = np.ascontiguousarray(de, np.float64)
    n, nr, nd = rho.size, re.size - 1, de.size - 1
    payload = struct.pack("<qiidii", n, rho_min, k, d_cut, nr, nd) + rho.tobytes() + delta.tobytes() + \
        re.tobytes() + de.tobytes()
    b = _run(exe, ["--decision"], payload)
    s1, s2, s3, count = struct.unpack("<iiiq", b[:20])
    o = 20
    ids = np.frombuffer(b, np.int32, k, o); o += 4 * k
    deltas = np.frombuffer(b, np.float64, k, o); o += 8 * k
    rhos = np.frombuffer(b, np.int32, k, o); o += 4 * k
    dmin, centers = struct.unpack("<dq", b[o:o + 16]); o += 16
    counts = np.frombuffer(b, np.int64, nr * nd, o).reshape(nr, nd)
    return {"status": (s1, s2, s3), "count": count, "ids": ids[:count], "deltas": deltas[:count],
            "rhos": rhos[:count], "delta_min": dmin, "centers": centers, "counts": counts}


def check(got, rho, delta, rho_min, k, d_cut, re, de, ctx=""):
    assert got["status"] == (0, 0, 0), ctx
    ids, dl, rh = D.top_delta(rho, delta, rho_min, k)
    assert got["count"] == ids.size, ctx
    assert np.array_equal(got["ids"], ids), ctx
    assert np.array_equal(got["deltas"].view(np.int64), dl.view(np.int64)), ctx
    assert np.array_equal(got["rhos"], rh), ctx
    dmin, cent = D.suggest_delta_min(dl, d_cut)
    if dmin is None:
        assert math.isnan(got["delta_min"]) and got["centers"] == 0, ctx
    else:
        assert got["delta_min"] == dmin and got["centers"] == cent, ctx
    assert np.array_equal(got["counts"], D.histogram(rho, delta, re, de)), ctx


def test_dpc_outputs(emu_exe):
    for d, seed in ((2, 1), (3, 2)):
        job = inputs.blob_job(70 + seed, 1500, d, 6, 400.0, 1500.0, 0.1)
        ex = dpc_oracle.dpc(job.pts, job.d_cut, job.rho_min, job.delta_min)
        re = [1, 5, 10, 20, 40, 80, 1e9]
        de = [0.0, job.d_cut / 4, job.d_cut / 2, job.d_cut, 2 * job.d_cut, 8 * job.d_cut, math.inf]
        for k in (1, 7, 64, 3000):
            k = min(k, 4096)
            got = run_decision_emu(emu_exe, ex["rho"], ex["delta"], job.rho_min, k, job.d_cut, re, de)
            check(got, ex["rho"], ex["delta"], job.rho_min, k, job.d_cut, re, de, (d, k))
        ax = approx_oracle.approx_dpc(job.pts, job.d_cut, job.rho_min, job.delta_min)  # many equal deltas
        got = run_decision_emu(emu_exe, ax["rho"], ax["delta"], job.rho_min, 500, job.d_cut, re, de)
        check(got, ax["rho"], ax["delta"], job.rho_min, 500, job.d_cut, re, de, ("approx", d))


def test_ties_zeros_and_noise(emu_exe):
    rng = np.random.default_rng(5)
    n = 5000
    rho = rng.integers(1, 6, n)
    delta = rng.integers(0, 4, n).astype(np.float64)  # heavy ties, zeros
    delta[[3, 77]] = math.inf
    re = np.arange(0, 7, dtype=np.float64)
    de = [0.0, 1.0, 2.0, 3.0]
    for k, rho_min in ((1, 1), (50, 2), (4096, 1), (300, 6)):  # rho_min 6: nobody qualifies
        got = run_decision_emu(emu_exe, rho, delta, rho_min, k, 0.5, re, de)
        check(got, rho, delta, rho_min, k, 0.5, re, de, (k, rho_min))


def test_large_bin_grid_uses_global_counts(emu_exe):
    rng = np.random.default_rng(6)
    n = 3000
    rho = rng.integers(1, 300, n)
    delta = rng.uniform(0, 1000, n)
    re = np.arange(0, 301, dtype=np.float64)        # 300 x 40 = 12000 bins: past the LDS histogram
    de = np.linspace(0, 1000, 41)
    got = run_decision_emu(emu_exe, rho, delta, 1, 10, 5.0, re, de)
    check(got, rho, delta, 1, 10, 5.0, re, de)
