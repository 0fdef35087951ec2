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
from tests import digests
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


@pytest.mark.parametrize("d", [3, 4])
def test_separate_calls_and_no_reuse(dpc, d):
    job = inputs.blob_job(77, 5000, d, 7, 500.0, 2000.0, 0.1)
    _say(f"separate calls d={d}")
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


def sum_rho_by_pair_count(job):
    """n + 2 * #{i < j : D2 < R}, counted by scipy's kd-tree (closed ball of radius
    sqrt(R - 1/2) holds exactly the integer D2 <= R - 1), independent of both paths."""
    from scipy.spatial import cKDTree
    R = dpc_oracle.cutoff_square(job.d_cut)
    tree = cKDTree(job.pts.astype(np.float64))
    return int(tree.count_neighbors(tree, math.sqrt(R - 0.5)))


def check_properties(job, out):
    """Properties that hold at any size (Defs. 1-6)."""
    rho, dep, delta, lab = out["rho"], out["dep"], out["delta"], out["label"]
    _say(f"{job.name}: sum of rho against the kd-tree pair count")
    assert int(rho.sum(dtype=np.int64)) == sum_rho_by_pair_count(job)
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


def check_sampled(job, out, n_rho, n_dep, seed=0):
    """Sampled points against the oracle computed one by one (localises a mismatch)."""
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
    assert np.array_equal(out["rho"][which], rho_s)
    assert np.array_equal(out["dep"][which][ok], dep_s[ok])
    assert np.array_equal(out["delta"][which][ok], scan.dependent_distance(d2_s[ok]))


def check_full_size(dpc, job, n_rho=1500, n_dep=160, seed=0):
    """Whole-output parity at full size: the outputs' digests against those of the
    oracle (tests/golden/oracle_digests.json, written by an oracle-only script),
    plus properties at any size.  On a digest mismatch, or without a digest, the
    sampled oracle check runs to localise the difference."""
    out = run_gpu(dpc, job.pts, job.d_cut, job.rho_min, job.delta_min)
    rec = digests.load().get(job.name)
    check_properties(job, out)
    if rec is None:
        _say(f"{job.name}: no oracle digest stored; sampled check only")
        check_sampled(job, out, n_rho, n_dep, seed)
        return out
    assert rec["input"] == digests.input_digest(job), "the stored digest belongs to other inputs"
    got = digests.output_digests(out)
    bad = [k for k in digests.OUT_KEYS if got[k] != rec[k]]
    if got["ncenters"] != rec["ncenters"]:
        bad.append("ncenters")
    if bad:
        _say(f"{job.name}: digests differ in {bad}; localising with the sampled oracle check")
        check_sampled(job, out, n_rho, n_dep, seed)
        raise AssertionError(f"{job.name}: whole-output digests differ from the oracle's in {bad}")
    _say(f"{job.name}: rho, dep, delta and labels equal the oracle's, all {job.n} points")
    return out


def test_blobs_1m_whole(dpc):
    check_full_size(dpc, inputs.blobs_1m())


def test_walks_4m_whole(dpc):
    check_full_size(dpc, inputs.walks_4m(), n_rho=1000, n_dep=40)


def test_reuse_grid_is_checked(dpc):
    """DPC_REUSE_GRID with a workspace that holds no grid of these inputs computes
    nothing (outputs untouched) and reports DPC_EINVAL; a reused grid keeps the
    out-of-range status of its build."""
    job = inputs.blob_job(81, 3000, 3, 5, 500.0, 2000.0, 0.05)
    t = torch.from_numpy(job.pts).cuda()
    n = job.n
    rho = dpc.dpc_density(t, job.d_cut)
    torch.cuda.synchronize()
    for case in ("fresh workspace", "other points", "other cut-off"):
        _say(f"reuse check: {case}")
        ws = dpc.workspace(n, job.d, job.d_cut)
        ws.zero_()
        pts = t
        if case != "fresh workspace":
            dpc.dpc_density(t.clone() if case == "other points" else t,
                            job.d_cut * (1.5 if case == "other cut-off" else 1.0), ws=ws)
            dpc.dpc_sync_status(ws)
        dep = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        delta = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
        dpc.dpc_dependent(pts, job.d_cut, rho, dep=dep, delta=delta, flags=dpc.DPC_REUSE_GRID, ws=ws)
        with pytest.raises(dpc.DpcError) as e:
            dpc.dpc_sync_status(ws)
        assert e.value.status == dpc.DPC_EINVAL, case
        assert (dep.cpu().numpy() == -7).all() and (delta.cpu().numpy() == -7.0).all(), case
    _say("reuse check: out-of-range status kept")
    bad = job.pts.copy()
    bad[5, 2] = 131072 + 77
    tb = torch.from_numpy(bad).cuda()
    ws = dpc.workspace(n, job.d, job.d_cut)
    rho_b = dpc.dpc_density(tb, job.d_cut, ws=ws)
    dep, delta = dpc.dpc_dependent(tb, job.d_cut, rho_b, flags=dpc.DPC_REUSE_GRID, ws=ws)
    with pytest.raises(dpc.DpcError) as e:
        dpc.dpc_sync_status(ws)
    assert e.value.status == dpc.DPC_ERANGE
    want = oracle_run(np.clip(bad, 0, 131071), job.d_cut, job.rho_min, job.delta_min)
    assert np.array_equal(rho_b.cpu().numpy(), want["rho"])
    assert np.array_equal(dep.cpu().numpy(), want["dep"])
    assert np.array_equal(delta.cpu().numpy().view(np.int64), want["delta"].view(np.int64))


@pytest.mark.parametrize("lanes", [1, 2])
def test_kernel_forms_single_job(dpc, lanes):
    """Both kernel forms (64-query tasks, one query per lane) on one job through a
    one-job batch with that option, against the oracle."""
    for d in (2, 3, 4, 6):
        job = inputs.blob_job(90 + d, 4000, d, 6, 500.0, 2500.0, 0.05)
        _say(f"kernel form {lanes}: d={d}")
        b = dpc.Batch([(torch.from_numpy(job.pts).cuda(), job.d_cut, job.rho_min, job.delta_min)],
                      [dpc.Tuning.make(lanes=lanes)])
        b.run()
        b.sync_status()
        got = {k: v.cpu().numpy() for k, v in b.out[0].items()}
        got["ncenters"] = int(got["ncenters"][0])
        b.close()
        compare(got, oracle_run(job.pts, job.d_cut, job.rho_min, job.delta_min), ctx=f"lanes={lanes} d={d}")
