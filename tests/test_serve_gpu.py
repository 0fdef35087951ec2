"""Served loop: every result in the mix equals the job run alone.

New-job requests must return the labels (and center count) that dpc_run gives
for the job alone; re-threshold requests must return the labels of dpc_label on
the job's own rho, dep and delta, which the oracle's labelling reproduces.  Run
once with a roomy HBM budget and once with a budget so small that jobs are
evicted and requests wait for memory.
"""
import sys

import numpy as np
import pytest

from oracle import scan
from paper_2207_04649_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2207_04649_amd import dpc, serve
    dpc.lib()
    return dpc, serve


def small_trace(seed, count=48):
    trace = inputs.serve_trace(rate=400.0, duration=count / 400.0 * 1.5, seed=seed, n_lo=300, n_hi=20_000)
    return trace[:count]


def alone(dpc, job_pts, d_cut, rho_min, delta_min):
    t = torch.from_numpy(job_pts).cuda()
    n, d = t.shape
    ws = dpc.workspace(n, d, d_cut)
    out = dpc.dpc_run(t, d_cut, rho_min, delta_min, ws=ws)
    dpc.dpc_sync_status(ws)
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("roomy,slots", [(True, 4), (False, 3)])
def test_served_results_equal_alone(mods, roomy, slots):
    dpc, serve = mods
    reqs = serve.trace_requests(small_trace(11), lambda spec: spec.make())
    # The tight budget holds the largest job (and its workspace) with a third to
    # spare, far less than all the jobs together, so jobs must be evicted.
    biggest = max(serve.Server.resident_bytes(*q.pts.shape) + dpc.dpc_workspace_bytes(*q.pts.shape, q.d_cut)
                  for q in reqs if q.kind == "new")
    budget = 64 << 30 if roomy else int(1.3 * biggest)
    _say(f"serving {len(reqs)} requests, budget {budget >> 20} MiB, {slots} slots")
    srv = serve.Server(budget_bytes=budget, slots=slots, relabel_slots=0 if slots == 3 else 1)
    srv.run(reqs)
    if not roomy:
        assert srv.stats["evicted"] > 0, "the small budget must force evictions"
    assert srv.peak_used <= budget
    by_key = {q.job_key: q for q in reqs if q.kind == "new"}
    cache = {}
    for q in reqs:
        assert q.t_done >= q.t_arrival
        if q.dropped:
            continue
        src = by_key[q.job_key]
        if q.job_key not in cache:
            cache[q.job_key] = alone(dpc, src.pts, src.d_cut, src.rho_min, src.delta_min)
        ref = cache[q.job_key]
        if q.kind == "new":
            assert np.array_equal(q.labels.numpy(), ref["label"]), f"request {q.rid}"
            assert int(q.ncenters[0]) == int(ref["ncenters"][0])
        else:
            lab, nc = scan.labels(ref["rho"], ref["dep"], ref["delta"], q.rho_min, q.delta_min)
            assert np.array_equal(q.labels.numpy(), lab), f"re-threshold {q.rid}"
            assert int(q.ncenters[0]) == nc
    summary = serve.latency_summary(reqs)
    _say(f"latency {summary}, stats {dict(srv.stats)}")
    assert summary["new"]["count"] == sum(1 for q in reqs if q.kind == "new")


def _make_job(spec):
    return spec.make()


def test_served_jobs_vs_oracle_digests(mods):
    """The serving trace with new jobs of up to 200,000 points (d 2..8): every new
    job's rho, dep, delta and labels against the oracle's digests (written by an
    oracle-only script), and every re-threshold's labels against the oracle's
    labelling of the job's (so verified) rho, dep and delta.  Re-thresholds run on
    their own slot."""
    import concurrent.futures as cf
    import multiprocessing as mp

    from tests import digests

    dpc, serve = mods
    rec = digests.load().get("serve_test")
    if rec is None:
        pytest.skip("no oracle digests stored for the serving trace")
    trace = inputs.serve_trace(**rec["trace"])
    specs = [r.spec for r in trace if r.kind == "new"]
    _say(f"drawing {len(specs)} served jobs")
    with cf.ProcessPoolExecutor(16, mp_context=mp.get_context("spawn")) as ex:
        jobs = dict(zip((sp.seed for sp in specs), ex.map(_make_job, specs, chunksize=2)))
    reqs = serve.trace_requests(trace, lambda spec: jobs[spec.seed])
    srv = serve.Server(budget_bytes=64 << 30, slots=4, relabel_slots=1, keep_outputs=True)
    _say(f"serving {len(reqs)} requests")
    srv.run(reqs)
    by_key = {}
    for q in reqs:
        if q.kind != "new":
            continue
        want = rec["jobs"][str(q.seed)]
        assert want["input"] == digests.input_digest(jobs[q.seed])[:16]
        got = {"rho": q.rho.numpy(), "dep": q.dep.numpy(), "delta": q.delta.numpy(), "label": q.labels.numpy(),
               "ncenters": int(q.ncenters[0])}
        dg = digests.output_digests(got, short=16)
        bad = [f for f in (*digests.OUT_KEYS, "ncenters") if dg[f] != want[f]]
        assert not bad, f"new job {q.rid} (seed {q.seed}, n={want['n']}, d={want['d']}): {bad} differ from the oracle"
        by_key[q.job_key] = got
    relabels = 0
    for q in reqs:
        if q.kind != "rethreshold" or q.dropped:
            continue
        src = by_key[q.job_key]
        lab, nc = scan.labels(src["rho"], src["dep"], src["delta"], q.rho_min, q.delta_min)
        assert np.array_equal(q.labels.numpy(), lab), f"re-threshold {q.rid}"
        assert int(q.ncenters[0]) == nc
        relabels += 1
    summary = serve.latency_summary(reqs)
    _say(f"{len(by_key)} new jobs and {relabels} re-thresholds equal the oracle; latency {summary}")
    assert relabels > 0
