"""Many problems in one launch per phase (dpc_batch_*), through the C ABI.

Every job of a batch must give, bit for bit, what the oracle gives for it alone
(rho, dep, labels, ncenters; delta to 0 ULP), and what dpc_run gives for it
alone; the batch must replay correctly from a captured HIP graph.
"""
import sys

import numpy as np
import pytest

from oracle import scan
from paper_2207_04649_amd import inputs
from tests import oracle_pins as pins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("rho", "dep", "delta", "label", "ncenters")


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


def to_host(out):
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["ncenters"] = int(res["ncenters"][0])
    return res


def single(dpc, pts_t, d_cut, rho_min, delta_min):
    n, d = pts_t.shape
    ws = dpc.workspace(n, d, d_cut)
    out = dpc.dpc_run(pts_t, d_cut, rho_min, delta_min, ws=ws)
    dpc.dpc_sync_status(ws)
    return to_host(out)


def mixed_jobs(seed=0, count=40):
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(count):
        d = int(rng.integers(1, 9))
        n = int(rng.choice([1, 2, 7, 63, 64, 65, 200, 777, 1500, 3000]))
        hi = int(rng.choice([50, 3000, 131071]))
        pts = inputs.uniform_points(n, d, hi, 1000 * seed + k)
        if k % 3 == 0 and n > 1:
            pts[n // 2:] = pts[: n - n // 2]
        d_cut = float(rng.choice([0.5, 1.0, 7.5, 40.0, 300.0, 2500.0, 20000.0]))
        jobs.append((pts, d_cut, int(rng.integers(1, 6)), d_cut * float(rng.uniform(1.01, 4.0))))
    return jobs


def run_batch(dpc, jobs, tunings=None):
    problems = [(torch.from_numpy(p).cuda(), dc, rm, dm) for p, dc, rm, dm in jobs]
    b = dpc.Batch(problems, tunings)
    b.run()
    b.sync_status()
    return b, problems, [to_host(o) for o in b.out]


def test_batch_small_mixed_vs_oracle(dpc):
    jobs = mixed_jobs(0)
    _say(f"batch of {len(jobs)} mixed jobs")
    b, _, outs = run_batch(dpc, jobs)
    for k, (job, got) in enumerate(zip(jobs, outs)):
        pins.assert_same(got, pins.run(scan, *job), keys=KEYS, ctx=f"job {k} n={job[0].shape} d_cut={job[1]}")
    b.close()


def test_batch_generator_jobs_vs_single_and_oracle(dpc):
    specs = inputs.batch_specs(64)
    jobs = [(j.pts, j.d_cut, j.rho_min, j.delta_min) for j in (s.make() for s in specs)]
    _say(f"batch of {len(jobs)} generator jobs, {sum(j[0].shape[0] for j in jobs)} points")
    b, problems, outs = run_batch(dpc, jobs)
    for k, ((pts_t, dc, rm, dm), got) in enumerate(zip(problems, outs)):
        pins.assert_same(got, single(dpc, pts_t, dc, rm, dm), keys=KEYS, ctx=f"job {k} vs dpc_run")
        if jobs[k][0].shape[0] <= 6000:
            pins.assert_same(got, pins.run(scan, *jobs[k]), keys=KEYS, ctx=f"job {k} vs oracle")
    b.close()


def test_batch_graph_replay(dpc):
    jobs = mixed_jobs(1, count=24)
    problems = [(torch.from_numpy(p).cuda(), dc, rm, dm) for p, dc, rm, dm in jobs]
    b = dpc.Batch(problems)
    b.run()
    b.sync_status()
    want = [to_host(o) for o in b.out]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            dpc.dpc_batch_run(b.handle, b.ws, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    for rep in range(3):
        for o in b.out:  # eager work between replays; a replay that does nothing fails
            for v in o.values():
                v.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        b.sync_status()
        for k, o in enumerate(b.out):
            pins.assert_same(to_host(o), want[k], keys=KEYS, ctx=f"replay {rep} job {k}")
    b.close()


def test_batch_rerun_and_tunings_agree(dpc):
    jobs = mixed_jobs(2, count=16)
    b, problems, first = run_batch(dpc, jobs)
    b.run()
    b.sync_status()
    for k, o in enumerate(b.out):
        pins.assert_same(to_host(o), first[k], keys=KEYS, ctx=f"rerun job {k}")
    b.close()
    tun = [dpc.Tuning.make(subdiv=1 + k % 4, strip_cells=(0, 3, 16)[k % 3],
                           stages=[((1, 1), (3, 4)), ((2, 1),), ((1, 1), (2, 2), (4, 8)), ((0, 1),),
                                   ((0, 1), (2, 4))][k % 5],
                           ring_cap=(0, 4, 300)[k % 3], grid_dims=(0, 2, 3, 8)[k % 4], lanes=(0, 1, 2)[k % 3])
           for k in range(len(jobs))]
    b2, _, tuned = run_batch(dpc, jobs, tun)
    for k in range(len(jobs)):
        pins.assert_same(tuned[k], first[k], keys=KEYS, ctx=f"tuned job {k}")
    b2.close()


def test_batch_device_errors_name_the_job(dpc):
    good = inputs.uniform_points(100, 2, 5000, 1)
    bad = good.copy()
    bad[3, 0] = -5
    jobs = [(good, 300.0, 1, 900.0), (bad, 300.0, 1, 900.0), (good, 300.0, 1, 900.0)]
    problems = [(torch.from_numpy(p).cuda(), dc, rm, dm) for p, dc, rm, dm in jobs]
    b = dpc.Batch(problems)
    b.run()
    with pytest.raises(dpc.DpcError) as e:
        b.sync_status()
    assert e.value.status == dpc.DPC_ERANGE and "job 1" in str(e.value)
    clamped = pins.run(scan, np.clip(bad, 0, 131071), 300.0, 1, 900.0)
    pins.assert_same(to_host(b.out[1]), clamped, keys=KEYS, ctx="clamped job")
    pins.assert_same(to_host(b.out[0]), pins.run(scan, good, 300.0, 1, 900.0), keys=KEYS, ctx="good job")
    b.close()


def _make_job(spec):
    return spec.make()


def test_batch4096_whole_vs_oracle_digests(dpc):
    """All 4096 jobs of the batch workload in one batch, every job's rho, dep,
    delta and labels against the digests of the oracle's outputs (written by an
    oracle-only script, tests/golden/make_oracle_digests.py)."""
    import multiprocessing as mp
    import concurrent.futures as cf

    from tests import digests

    rec = digests.load().get("batch4096")
    if rec is None:
        pytest.skip("no oracle digests stored for the 4096-job batch")
    specs = inputs.batch_specs(rec["count"])
    _say(f"drawing {len(specs)} batch jobs")
    with cf.ProcessPoolExecutor(16, mp_context=mp.get_context("spawn")) as ex:
        made = list(ex.map(_make_job, specs, chunksize=16))
    jobs = [(j.pts, j.d_cut, j.rho_min, j.delta_min) for j in made]
    _say(f"batch of {len(jobs)} jobs, {sum(j[0].shape[0] for j in jobs)} points")
    b, _, outs = run_batch(dpc, jobs)
    bad = []
    for k, (job, got, want) in enumerate(zip(made, outs, rec["jobs"])):
        assert want["seed"] == specs[k].seed and want["input"] == digests.input_digest(job)[:16]
        dg = digests.output_digests(got, short=16)
        if any(dg[f] != want[f] for f in (*digests.OUT_KEYS, "ncenters")):
            bad.append(k)
    b.close()
    if bad:
        k = bad[0]
        _say(f"{len(bad)} jobs differ from the oracle digests; localising job {k}")
        pins.assert_same(outs[k], pins.run(scan, *jobs[k]), keys=KEYS, ctx=f"job {k}")
    assert not bad, f"{len(bad)} of {len(jobs)} jobs differ from the oracle (first {bad[:10]})"
