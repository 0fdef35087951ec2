"""Parity of the HIP path (through the C ABI) with the oracle.

rho, dep and labels must match bit for bit, and delta to 0 ULP (it is the
correctly rounded square root of the same exact integer), on the same seeded
inputs.  Small inputs are compared whole; the full-size workloads on samples
the oracle computes one by one, plus properties that hold at any size.
"""
import math
import sys

import numpy as np
import pytest

from oracle import dpc_oracle, scan
from paper_2207_04649_amd import inputs
from tests import oracle_pins as pins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_04649_amd import dpc as binding
    binding.lib()
    return binding


def run_gpu(dpc, pts, d_cut, rho_min, delta_min, separate=False, reuse=True):
    t = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.int32)).cuda()
    n, d = t.shape
    ws = dpc.workspace(n, d, d_cut)
    if separate:
        rho = dpc.dpc_density(t, d_cut, ws=ws)
        dep, delta = dpc.dpc_dependent(t, d_cut, rho, flags=dpc.DPC_REUSE_GRID if reuse else 0, ws=ws)
        label, nc = dpc.dpc_label(rho, dep, delta, rho_min, delta_min, ws=ws)
        out = {"rho": rho, "dep": dep, "delta": delta, "label": label, "ncenters": nc}
    else:
        out = dpc.dpc_run(t, d_cut, rho_min, delta_min, ws=ws)
    dpc.dpc_sync_status(ws)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["ncenters"] = int(res["ncenters"][0])
    return res


def oracle_run(pts, d_cut, rho_min, delta_min):
    return pins.run(scan, pts, d_cut, rho_min, delta_min)


def compare(got, want, ctx=""):
    for k in ("rho", "dep", "label"):
        a = np.asarray(got[k], np.int64)
        b = np.asarray(want[k], np.int64)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} points, first {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    a = np.asarray(got["delta"], np.float64).view(np.int64)
    b = np.asarray(want["delta"], np.float64).view(np.int64)
    assert np.array_equal(a, b), f"{ctx}: delta differs at {np.count_nonzero(a != b)} points"
    assert got["ncenters"] == want["ncenters"], ctx


def test_hand_example(dpc):
    import json
    g = json.load(open(pins.GOLDEN))
    P = np.array(g["points"], np.int32)
    for case in g["cases"]:
        for lc in case["labels"]:
            _say(f"hand example d_cut={case['d_cut']} {lc}")
            out = run_gpu(dpc, P, case["d_cut"], lc["rho_min"], lc["delta_min"])
            assert out["rho"].tolist() == case["rho"]
            assert out["dep"].tolist() == case["dep"]
            assert out["label"].tolist() == lc["label"]
            if "delta" in case:
                assert out["delta"].tolist() == case["delta"]


SMALL = []
for _seed in range(3):
    for _d in range(1, 9):
        for _n, _hi, _dc in [(1, 10, 2.0), (2, 3, 1.5), (65, 30, 6.0), (700, 60, 9.5),
                             (1500, 5000, 700.0), (2000, 100_000, 9000.0)]:
            SMALL.append((_seed, _d, _n, _hi, _dc))


@pytest.mark.parametrize("seed,d,n,hi,d_cut", SMALL)
def test_random_small(dpc, seed, d, n, hi, d_cut):
    _say(f"random seed={seed} d={d} n={n} hi={hi} d_cut={d_cut}")
    pts = inputs.uniform_points(n, d, hi, 7919 * seed + 101 * d + n)
    rho_min, delta_min = 2, d_cut * 1.7
    compare(run_gpu(dpc, pts, d_cut, rho_min, delta_min), oracle_run(pts, d_cut, rho_min, delta_min),
            ctx=f"seed={seed} d={d} n={n}")


@pytest.mark.parametrize("d", [1, 2, 3, 4, 6, 8])
def test_blob_jobs(dpc, d):
    job = inputs.blob_job(600 + d, 3000, d, 6, 500.0, 2500.0, 0.05)
    _say(f"blob job d={d} d_cut={job.d_cut}")
    compare(run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min),
            oracle_run(job.pts, job.d_cut, job.rho_min, job.delta_min), ctx=f"blob d={d}")


@pytest.mark.parametrize("d_cut", [0.5, 1.0, 1.0000001, 2.0, 99.5, 3000.0, 12000.0, 40000.0, 200000.0])
def test_cutoff_extremes(dpc, d_cut):
    """Tiny cut-offs (R = 1: duplicates only), large ones (exact int64 path) and one
    beyond every distance (every density n)."""
    pts = inputs.uniform_points(900, 2, 3000, 31)
    pts[::7] = pts[1::7][: pts[::7].shape[0]]  # duplicates
    _say(f"cutoff extreme d_cut={d_cut}")
    compare(run_gpu(dpc, pts, d_cut, 1, d_cut * 1.01 + 1), oracle_run(pts, d_cut, 1, d_cut * 1.01 + 1),
            ctx=f"d_cut={d_cut}")


def test_cell_boundaries_and_threshold_pairs(dpc):
    """Points on multiples of the cell side, and pairs at D2 = R - 1, R, R + 1."""
    d_cut = 200.0
    L = dpc.dpc_plan(10, 2, d_cut)["cell_side"]
    rng = np.random.default_rng(5)
    base = rng.integers(1, 400, size=(300, 2)) * L
    pairs = []
    for off in [(120, 160), (199, 19), (0, 200), (200, 0), (141, 141), (199, 20)]:  # D2 = 40000 +- small
        for b in base[:40]:
            pairs.append(b + np.array(off))
    pts = np.concatenate([base, np.array(pairs), base[:50] + 1, base[:50] - 1]).astype(np.int32)
    pts = np.clip(pts, 0, 131071).astype(np.int32)
    _say("cell boundaries")
    compare(run_gpu(dpc, pts, d_cut, 2, 450.0), oracle_run(pts, d_cut, 2, 450.0), ctx="boundaries")


def test_lattice_ties(dpc):
    """Every point has many equidistant neighbours of equal density."""
    for d, side, sp, dc in [(2, 40, 7, 7.0), (2, 40, 7, 7.01), (3, 12, 5, 8.7), (1, 500, 3, 3.0)]:
        pts = inputs.lattice_points(side, d, sp, offset=3)
        _say(f"lattice d={d} side={side}")
        compare(run_gpu(dpc, pts, dc, 1, dc * 2), oracle_run(pts, dc, 1, dc * 2), ctx=f"lattice d={d}")


def test_separate_calls_and_no_reuse(dpc):
    job = inputs.blob_job(77, 5000, 3, 7, 500.0, 2000.0, 0.1)
    _say("separate calls")
    want = oracle_run(job.pts, job.d_cut, job.rho_min, job.delta_min)
    compare(run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min, separate=True), want, "reuse")
    compare(run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min, separate=True, reuse=False), want,
            "no reuse")


def test_rethreshold_labels(dpc):
    """Labels depend on (rho, dep, delta) and the thresholds only (decision graph)."""
    job = inputs.blob_job(78, 6000, 2, 9, 400.0, 1500.0, 0.1)
    t = torch.from_numpy(job.pts).cuda()
    ws = dpc.workspace(job.n, job.d, job.d_cut)
    out = dpc.dpc_run(t, job.d_cut, job.rho_min, job.delta_min, ws=ws)
    rho_o = scan.local_density(job.pts, job.d_cut)
    dep_o, d2_o = scan.dependent(job.pts, rho_o)
    delta_o = scan.dependent_distance(d2_o)
    for rm, dm in [(1, job.d_cut * 1.5), (5, job.d_cut * 3), (40, job.d_cut * 10), (1000, job.d_cut * 2)]:
        _say(f"rethreshold rho_min={rm} delta_min={dm}")
        lab, nc = dpc.dpc_label(out["rho"], out["dep"], out["delta"], rm, dm, ws=ws)
        want, nc_o = scan.labels(rho_o, dep_o, delta_o, rm, dm)
        assert np.array_equal(lab.cpu().numpy(), want)
        assert int(nc.item()) == nc_o


def test_deterministic(dpc):
    job = inputs.blob_job(79, 20000, 2, 10, 300.0, 1500.0, 0.05)
    _say("determinism")
    a = run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min)
    b = run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min)
    for k in ("rho", "dep", "delta", "label"):
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_out_of_range_coordinates_flagged(dpc):
    pts = inputs.uniform_points(500, 2, 131071, 3)
    bad = pts.copy()
    bad[3, 0] = -5
    bad[10, 1] = 131072 + 9
    t = torch.from_numpy(bad).cuda()
    ws = dpc.workspace(500, 2, 3000.0)
    _say("out of range")
    out = dpc.dpc_run(t, 3000.0, 2, 4000.0, ws=ws)
    with pytest.raises(dpc.DpcError) as e:
        dpc.dpc_sync_status(ws)
    assert e.value.status == dpc.DPC_ERANGE
    dpc.dpc_sync_status(ws)  # the flag was cleared
    clamped = np.clip(bad, 0, 131071)
    got = {k: v.cpu().numpy() for k, v in out.items()}
    got["ncenters"] = int(got["ncenters"][0])
    compare(got, oracle_run(clamped, 3000.0, 2, 4000.0), ctx="clamped")


def test_blobs_20k_full(dpc):
    job = inputs.blobs_20k()
    _say("blobs_20k full parity")
    compare(run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min),
            oracle_run(job.pts, job.d_cut, job.rho_min, job.delta_min), ctx="blobs_20k")


def check_full_size(dpc, job, n_rho=1500, n_dep=160, seed=0):
    """Full-size run checked on samples the oracle computes one by one, and on
    properties that hold at any size."""
    out = run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min)
    rng = np.random.default_rng(seed)
    n = job.n
    which = np.sort(rng.choice(n, size=min(n, n_rho), replace=False))
    _say(f"{job.name}: oracle densities of {which.size} samples")
    assert np.array_equal(out["rho"][which], scan.local_density_of(job.pts, job.d_cut, which))
    # the densest points and the points without a dependent are checked too
    top = np.argsort(-out["rho"], kind="stable")[:8]
    which = np.unique(np.concatenate([rng.choice(n, size=min(n, n_dep), replace=False), top]))
    _say(f"{job.name}: oracle dependents of {which.size} samples")
    rho_s, dep_s, d2_s = scan.dependent_of(job.pts, job.d_cut, which, max_walk=400)
    ok = dep_s != -2
    assert ok.sum() >= 0.8 * which.size
    assert np.array_equal(out["rho"][which], rho_s)
    assert np.array_equal(out["dep"][which][ok], dep_s[ok])
    assert np.array_equal(out["delta"][which][ok], scan.dependent_distance(d2_s[ok]))
    # properties at any size
    rho, dep, delta, lab = out["rho"], out["dep"], out["delta"], out["label"]
    assert np.count_nonzero(dep < 0) == 1
    i = np.nonzero(dep >= 0)[0]
    j = dep[i]
    higher = (rho[j] > rho[i]) | ((rho[j] == rho[i]) & (j < i))
    assert higher.all(), "every dependent point ranks higher"
    p = job.pts.astype(np.int64)
    d2 = np.sum((p[i] - p[j]) ** 2, axis=1)
    assert np.array_equal(np.sqrt(d2.astype(np.float64)), delta[i]), "delta = sqrt of the exact D2"
    assert math.isinf(delta[dep < 0][0])
    noise = rho < job.rho_min
    center = ~noise & (delta >= job.delta_min)
    assert ((lab == -1) == noise).all()
    assert (lab[center] == np.nonzero(center)[0]).all()
    other = ~noise & ~center
    assert (lab[other] == lab[dep[other]]).all()
    assert out["ncenters"] == int(center.sum())
    lab_o, nc_o = scan.labels(rho, dep, delta, job.rho_min, job.delta_min)
    assert np.array_equal(lab, lab_o) and nc_o == out["ncenters"]
    return out


def test_blobs_1m_sampled(dpc):
    check_full_size(dpc, inputs.blobs_1m())


def test_walks_4m_sampled(dpc):
    check_full_size(dpc, inputs.walks_4m(), n_rho=1000, n_dep=40)
