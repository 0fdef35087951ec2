#!/usr/bin/env python3
"""Write tests/golden/oracle_digests.json: digests of the C oracle's outputs.

Runs the plain O(n^2) oracle (oracle/scan.c, the straightforward algorithm of
Section 2.2 for Definitions 1-6) on the CPU for workloads too large to run it
inside a test, and stores SHA-256 digests of its rho, dep, delta and labels
(canonical bytes, see tests/digests.py).  It calls only ``oracle/`` and the
seeded generators of ``paper_2207_04649_amd.inputs``; no value comes from the
HIP library.

    python tests/golden/make_oracle_digests.py blobs_1m_d2 batch4096 walks_4m_d4

Workloads (each entry is rewritten when its run ends):

* blobs_20k_d2, blobs_1m_d2, walks_4m_d4: the single-job workloads;
* batch4096: every job of the 4096-job batch workload (job k drawn from seed
  4,000,000 + k), one record per job;
* serve_test: every new job of the served-workload trace the serving test
  replays (inputs.serve_trace with n up to 200,000, see SERVE_TEST), by seed.

Times: about 10 minutes for blobs_1m_d2 and 15 for batch4096 on 8 cores; the
4M-point 4-D workload takes hours (1.6e13 + 8e12 distance evaluations).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import scan  # noqa: E402
from paper_2207_04649_amd import inputs  # noqa: E402
from tests import digests  # noqa: E402

SINGLE = ("blobs_20k_d2", "blobs_1m_d2", "walks_4m_d4")
# the trace of the serving test: Poisson arrivals at 200 jobs/s for one second,
# new jobs with n log-uniform in [1000, 200000], d in 2..8
SERVE_TEST = {"rate": 200.0, "duration": 1.0, "seed": 5, "n_hi": 200_000}


def log(msg: str) -> None:
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def oracle_outputs(job) -> dict:
    rho = scan.local_density(job.pts, job.d_cut)
    dep, d2 = scan.dependent(job.pts, rho)
    delta = scan.dependent_distance(d2)
    label, nc = scan.labels(rho, dep, delta, job.rho_min, job.delta_min)
    return {"rho": rho, "dep": dep, "delta": delta, "label": label, "ncenters": nc, "d2": d2}


def run_single(name: str, save_dir: str | None) -> dict:
    job = inputs.WORKLOADS[name]()
    log(f"{name}: n={job.n} d={job.d} d_cut={job.d_cut}: oracle on {scan.threads()} threads")
    t0 = time.perf_counter()
    out = oracle_outputs(job)
    secs = time.perf_counter() - t0
    rec = digests.output_digests(out)
    rec.update({"input": digests.input_digest(job), "n": job.n, "d": job.d, "d_cut": job.d_cut,
                "rho_min": job.rho_min, "delta_min": job.delta_min, "sum_rho": int(out["rho"].sum(dtype=np.int64)),
                "oracle_seconds": round(secs, 1), "oracle_threads": scan.threads()})
    if save_dir:
        os.makedirs(save_dir, exist_ok=True)
        np.savez(os.path.join(save_dir, f"{name}.npz"), **{k: out[k] for k in ("rho", "dep", "d2", "label")})
    log(f"{name}: done in {secs:.0f} s, {rec['ncenters']} centers")
    return rec


def _make(spec):
    return spec.make()


def run_batch(count: int, workers: int) -> dict:
    specs = inputs.batch_specs(count)
    log(f"batch{count}: {count} jobs, {sum(s.n for s in specs)} points")
    recs = []
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers) as ex:
        for k, job in enumerate(ex.map(_make, specs, chunksize=8)):
            out = oracle_outputs(job)
            rec = digests.output_digests(out, short=16)
            rec.update({"seed": specs[k].seed, "n": job.n, "d": job.d, "input": digests.input_digest(job)[:16]})
            recs.append(rec)
            if (k + 1) % 256 == 0:
                log(f"batch{count}: {k + 1} jobs")
    secs = time.perf_counter() - t0
    return {"count": count, "jobs": recs, "oracle_seconds": round(secs, 1), "oracle_threads": scan.threads()}


def run_serve_test(workers: int) -> dict:
    trace = inputs.serve_trace(**SERVE_TEST)
    specs = [r.spec for r in trace if r.kind == "new"]
    log(f"serve_test: {len(trace)} requests, {len(specs)} new jobs, {sum(s.n for s in specs)} points")
    recs = {}
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers) as ex:
        for spec, job in zip(specs, ex.map(_make, specs, chunksize=2)):
            out = oracle_outputs(job)
            rec = digests.output_digests(out, short=16)
            rec.update({"n": job.n, "d": job.d, "input": digests.input_digest(job)[:16]})
            recs[str(spec.seed)] = rec
    secs = time.perf_counter() - t0
    return {"trace": SERVE_TEST, "jobs": recs, "oracle_seconds": round(secs, 1), "oracle_threads": scan.threads()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+", help=f"any of {SINGLE}, batch4096 and serve_test")
    ap.add_argument("--workers", type=int, default=4, help="processes drawing the batch jobs")
    ap.add_argument("--save-dir", default=None, help="also keep the oracle's arrays here (.npz)")
    args = ap.parse_args()
    scan.build(force=False)
    for name in args.workloads:
        if name in SINGLE:
            rec = run_single(name, args.save_dir)
        elif name.startswith("batch"):
            rec = run_batch(int(name[len("batch"):]), args.workers)
        elif name == "serve_test":
            rec = run_serve_test(args.workers)
        else:
            raise SystemExit(f"unknown workload {name}")
        data = digests.load()
        data[name] = rec
        digests.save(data)
        log(f"{name}: written to {digests.DIGEST_FILE}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
