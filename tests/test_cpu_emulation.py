"""The library's kernel sources run on the CPU (no GPU): every GPU thread is a
fiber and wave intrinsics are lockstep rendezvous (tests/cpu_emu).  This checks
the kernels' logic, termination and memory bounds (AddressSanitizer) against the
oracle before anything runs on a GPU.  It does not model the GPU's compiler or
memory system."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import scan
from paper_2207_04649_amd import inputs
from tests import oracle_pins as pins
from tests.cpu_emu import build_emu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu_exe():
    return build_emu.build(os.path.join(ROOT, "_build", "emu"), asan=True)


def _record(pts, d_cut, rho_min, delta_min):
    pts = np.ascontiguousarray(pts, np.int32)
    n, d = pts.shape
    return struct.pack("<qidid", n, d, float(d_cut), int(rho_min), float(delta_min)) + pts.tobytes()


def _parse(b, o, n):
    st, st2, nc = struct.unpack("<iiq", b[o:o + 16])
    o += 16
    out = {"status": st, "sync": st2, "ncenters": nc}
    for k, dt, sz in (("rho", np.int32, 4), ("dep", np.int32, 4), ("delta", np.float64, 8), ("label", np.int32, 4)):
        out[k] = np.frombuffer(b, dt, n, o).copy()
        o += sz * n
    return out, o


def _run(exe, args, payload, extra_env=None):
    with tempfile.TemporaryDirectory() as tmp:
        fin, fout = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
        with open(fin, "wb") as f:
            f.write(payload)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0", **(extra_env or {}))
        r = subprocess.run([exe, *args, fin, fout], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stderr[-3000:]
        return open(fout, "rb").read()


def run_emu(exe, pts, d_cut, rho_min, delta_min, extra_env=None):
    b = _run(exe, [], _record(pts, d_cut, rho_min, delta_min), extra_env)
    return _parse(b, 0, int(np.asarray(pts).shape[0]))[0]


def run_emu_batch(exe, jobs, tuning=None):
    """jobs: list of (pts, d_cut, rho_min, delta_min), run through the batch entry points
    (every job with the plan options of the driver's --tuning spec, if given)."""
    payload = struct.pack("<i", len(jobs)) + b"".join(_record(*j) for j in jobs)
    b = _run(exe, ["--batch"] + (["--tuning", tuning] if tuning else []), payload)
    outs, o = [], 0
    for j in jobs:
        out, o = _parse(b, o, int(np.asarray(j[0]).shape[0]))
        outs.append(out)
    return outs


# The dense cell table spans the whole coordinate domain, so the cut-offs here keep
# it small enough for an emulated fill and scan (both the 16-bit and int64 paths run).
CASES = [(seed, d, n, dc) for seed in range(2)
         for d, dc, ns in [(1, 40.0, (3, 900)), (2, 300.0, (1, 200, 900)), (2, 3000.0, (200,)),
                           (3, 2000.0, (200,)), (4, 4500.0, (150,)), (6, 14000.0, (40,)), (8, 27000.0, (12,))]
         for n in ns]


@pytest.mark.parametrize("seed,d,n,d_cut", CASES)
def test_emulated_kernels_match_oracle(emu_exe, seed, d, n, d_cut):
    pts = inputs.uniform_points(n, d, 131071, 31 * seed + 7 * d + n)
    if seed == 1:  # clustered copies: duplicates and many equal densities
        pts[n // 2:] = pts[: n - n // 2] + (pts[: n - n // 2] % 3)
        pts = np.clip(pts, 0, 131071).astype(np.int32)
    got = run_emu(emu_exe, pts, d_cut, 2, d_cut * 1.7)
    assert got["status"] == 0 and got["sync"] == 0
    pins.assert_same(got, pins.run(scan, pts, d_cut, 2, d_cut * 1.7), keys=("rho", "dep", "delta", "label", "ncenters"),
                     ctx=f"seed={seed} d={d} n={n}")


def test_emulated_blob_job(emu_exe):
    job = inputs.blob_job(12345, 2500, 2, 6, 500.0, 2000.0, 0.05)
    got = run_emu(emu_exe, job.pts, job.d_cut, job.rho_min, job.delta_min)
    pins.assert_same(got, pins.run(scan, job.pts, job.d_cut, job.rho_min, job.delta_min),
                     keys=("rho", "dep", "delta", "label", "ncenters"), ctx="blob job")


def test_emulated_out_of_range_is_flagged_and_bounded(emu_exe):
    pts = inputs.uniform_points(300, 3, 131071, 4)
    pts[5, 1] = -17
    pts[9, 2] = 131072 + 5000
    got = run_emu(emu_exe, pts, 2500.0, 1, 4000.0)
    assert got["status"] == 0 and got["sync"] == -2
    pins.assert_same(got, pins.run(scan, np.clip(pts, 0, 131071), 2500.0, 1, 4000.0),
                     keys=("rho", "dep", "delta", "label"), ctx="clamped")


def test_emulated_batch_matches_oracle(emu_exe):
    """Jobs of several dimensions and sizes (one of a single point) in one batch."""
    jobs = []
    for k, (n, d, dc) in enumerate([(200, 2, 3000.0), (1, 3, 100.0), (333, 1, 40.0), (150, 4, 9000.0),
                                    (90, 2, 300.0), (40, 6, 20000.0), (12, 8, 30000.0), (257, 3, 5000.0)]):
        pts = inputs.uniform_points(n, d, 131071, 900 + k)
        if k % 2:  # duplicates and equal densities
            pts[n // 2:] = pts[: n - n // 2]
        jobs.append((pts, dc, 2, dc * 1.7))
    jobs.append((inputs.blob_job(777, 600, 2, 4, 500.0, 2000.0, 0.05).pts, 900.0, 5, 5000.0))
    outs = run_emu_batch(emu_exe, jobs)
    for k, (job, got) in enumerate(zip(jobs, outs)):
        assert got["status"] == 0 and got["sync"] == 0, k
        pins.assert_same(got, pins.run(scan, *job), keys=("rho", "dep", "delta", "label", "ncenters"), ctx=f"job {k}")


def test_emulated_open_stage_hand_over_matches_oracle():
    """The lane form's open-point stage gives a point up to the ring search once a
    lane passes its candidate cap; with a cap of two candidates nearly every open
    point is handed over, and the results still equal the oracle's."""
    exe = build_emu.build(os.path.join(ROOT, "_build", "emu_cap"), asan=True, defines=("-DDPC_OPEN_CAP=2",))
    jobs = []
    for k, (n, d, dc) in enumerate([(400, 4, 12000.0), (300, 3, 9000.0), (200, 2, 4000.0)]):
        pts = inputs.uniform_points(n, d, 131071, 700 + k)
        pts[n // 2:] = pts[: n - n // 2] + (pts[: n - n // 2] % 7)
        jobs.append((np.clip(pts, 0, 131071).astype(np.int32), dc, 2, dc * 1.5))
    outs = run_emu_batch(exe, jobs, "lanes=2;open=2")
    for k, (job, got) in enumerate(zip(jobs, outs)):
        assert got["status"] == 0 and got["sync"] == 0, k
        pins.assert_same(got, pins.run(scan, *job), keys=("rho", "dep", "delta", "label", "ncenters"), ctx=f"job {k}")


@pytest.mark.parametrize("tuning", [
    "stages=0:1",                      # ball stage, ring search from nothing
    "stages=0:1,2:4;gm=2",             # ball then a gathered stage, partial grid
    "stages=1:1,3:4;subdiv=3",
    "lanes=2",                         # one query per lane, every dimension
    "lanes=2;stages=2:1;gm=2",         # lane form, radius-2 stage, partial grid
    "lanes=2;subdiv=2;ring=3",
    "lanes=2;open=2",                  # lane form with the open-point stage (line path)
    "lanes=2;open=3;ring=2",           # a radius-3 open-point stage (row path), short rings
    "lanes=1",                         # tasks of 64 queries, every dimension
])
def test_emulated_plan_options_match_oracle(emu_exe, tuning):
    jobs = []
    for k, (n, d, dc) in enumerate([(300, 2, 4000.0), (200, 4, 12000.0), (150, 3, 9000.0), (60, 6, 25000.0)]):
        pts = inputs.uniform_points(n, d, 131071, 500 + k)
        pts[n // 2:] = pts[: n - n // 2] + (pts[: n - n // 2] % 5)
        jobs.append((np.clip(pts, 0, 131071).astype(np.int32), dc, 2, dc * 1.5))
    outs = run_emu_batch(emu_exe, jobs, tuning)
    for k, (job, got) in enumerate(zip(jobs, outs)):
        assert got["status"] == 0 and got["sync"] == 0, (tuning, k)
        pins.assert_same(got, pins.run(scan, *job), keys=("rho", "dep", "delta", "label", "ncenters"),
                         ctx=f"{tuning} job {k}")
