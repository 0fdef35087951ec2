#!/usr/bin/env python3
"""End-to-end exact density-peaks clustering throughput on one MI355X.

One step = dpc_run on the resident input: grid build, local density (Def. 1),
density-rank sort, dependent point and distance (Defs. 2-3) and labels (Defs.
4-6), i.e. every step of the hot path.  The default workload is the
4,000,000-point 4-D random-walk set (100 reflecting walks with N(0, 500^2)
steps plus 2% uniform noise, int32 coordinates in [0, 100000], d_cut = 1500,
rho_min = 30, delta_min = 8000); ``--extra`` adds a shorter run of a second
workload (default the 1,000,000-point 2-D blob set) as an extra key.

Prints one JSON line: points/s, the roofline of the dominant kernel group and
of every group (timed with HIP events on the library's stream inside the timed
region), the kernels' candidate-test counts, and the oracle's CPU throughput on
a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and chip counts used for the rooflines.
HBM_PEAK_GBS = 8000.0
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_GHZ / 1000.0  # 32-bit lane-ops/s, in T


# A distance test of two d-dimensional points costs 2d + 2 32-bit lane ops in a
# plain form (a subtract and a multiply-add per dimension, a compare and a
# count or select).  Rates of tests in those ops, against the chip's 32-bit
# VALU peak, give the ALU rooflines.
def test_ops(d: int) -> int:
    return 2 * d + 2


def grid_bytes(n: int, d: int, cells: int) -> int:
    """Algorithmic HBM bytes of the grid build (a counting sort into cells): read the
    coordinates (4d per point) for the keys, write key and slot (8), read them and write
    the id and position (16), read the id and the coordinates and write the cell-order
    coordinates and their packed copy (4 + 8d + 4 ceil(d/2)); the cell table is zeroed,
    read and written by the scan (12 per cell)."""
    w = (d + 1) // 2
    return n * (4 * d + 8 + 16 + 4 + 8 * d + 4 * w) + 12 * (cells + 1)


def rooflines(job, per_ms: dict, sum_rho: int, work: dict, plan: dict) -> dict:
    """Roofline of each kernel group:

    * density (ALU): the algorithmic work is sum(rho), the in-ball tests no exact
      method can skip (Def. 1), each at test_ops(d);
    * search, peaks (ALU): the candidate tests each makes (counted by the kernels
      in an instrumented call), at test_ops(d): the pairs of a point and a point of
      higher rank in its searched cells (Defs. 2-3);
    * ringk (HBM): its candidates are scattered records (one wave per point reads
      the cells of a sparse annulus), so the bound is memory; the algorithmic
      bytes are the candidate records it must read, tests x record size (16-byte
      packed records in lane form with packed coordinates, else the rank key
      and the coordinate row);
    * finish (HBM): per point the cell-order position, best key and rank key
      read, dep, delta and rho written (36 bytes);
    * grid_build (HBM): grid_bytes() against 8 TB/s.
    """
    ops = test_ops(job.d)
    out = {}

    def alu(name, tests, algorithmic):
        t = per_ms.get(name)
        if not t:
            return
        a = tests * ops / (t * 1e-3) / 1e12
        out[name] = {"avg_ms": t, "bound": "alu", "achieved": a, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": a / VALU_PEAK_TOPS, "traffic": kernel_traffic(name, job.name),
                     "tests_per_launch": tests, "ops_per_test": ops, "work": algorithmic}

    alu("density", sum_rho, "sum of rho (in-ball pairs, self included)")
    alu("search", work.get("tests_search", 0), "candidate tests of the window search")
    alu("peaks", work.get("tests_peaks", 0), "candidate tests of the prefix scan")

    def hbm(name, nbytes, algorithmic):
        t = per_ms.get(name)
        if not t:
            return
        a = nbytes / (t * 1e-3) / 1e9
        out[name] = {"avg_ms": t, "bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": a / HBM_PEAK_GBS, "traffic": kernel_traffic(name, job.name),
                     "bytes_per_launch": nbytes, "work": algorithmic}

    packed = plan.get("lanes") and job.d <= 4 and plan.get("mode") == 0
    rec = 16 if packed else 8 + 4 * job.d
    hbm("ringk", work.get("tests_ring", 0) * rec, f"candidate records read ({rec} bytes per test)")
    hbm("finish", 36 * job.n, "36 bytes per point (position, best key, rank key in; dep, delta, rho out)")
    t = per_ms.get("grid_build")
    if t:
        b = grid_bytes(job.n, job.d, plan["cells"])
        a = b / (t * 1e-3) / 1e9
        out["grid_build"] = {"avg_ms": t, "bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": a / HBM_PEAK_GBS, "traffic": kernel_traffic("grid_build", job.name),
                             "bytes_per_launch": b}
    return out


# HBM bytes per launch of the kernel groups, from two rocprofv3 --pmc runs of this
# script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# counter reads for a plain copy of known size in the same run (see
# paper_2207_04649_amd/prof_summary.py hbm).  The figures belong to the kernel
# sources they were taken with: when those change, traffic is reported as null.
KERNEL_SOURCES = ("paper_2207_04649_amd/csrc/density.hip", "paper_2207_04649_amd/csrc/dependent.hip",
                  "paper_2207_04649_amd/csrc/grid.hip", "paper_2207_04649_amd/csrc/tasks.h",
                  "paper_2207_04649_amd/csrc/common.h", "paper_2207_04649_amd/csrc/api.hip",
                  "paper_2207_04649_amd/csrc/label.hip")
# The kernels of each timed group (one step of dpc_run), for summing their counters.
GROUP_KERNELS = {
    "grid_build": ("k_stamp_grid", "k_fill_u32", "k_cell_keys", "k_scan_tiles", "k_scan_sums", "k_scan_add",
                   "k_scatter", "k_gather_pts", "k_strip_count", "k_strip_tasks", "k_zero_count"),
    "density": ("k_density", "k_density_lanes"),
    "rank_sort": ("k_rank_hist", "k_rank_scatter"),
    "search": ("k_search", "k_search_lanes", "k_collect"),
    "open_search": ("k_search_open",),
    "ringk": ("k_ringk",),
    "peaks": ("k_rank_gather", "k_peaks"),
    "finish": ("k_finish",),
    "label": ("k_label_init", "k_jump", "k_root"),
}
# The counters of profiles/hbm_counters_<workload>.txt (groups whose kernels run
# only in them; k_jump runs 3 times per step).
HBM_BYTES: dict = {  # {workload: {"source": hash, group: bytes per launch}}
    "walks_4m_d4": {"source": "609bf7a7ba72f254", "ringk": 4757.5e6, "search": (1058.3 + 5.0) * 1e6,
                    "density": 889.7e6, "finish": 1044.2e6, "peaks": (45.2 + 42.7) * 1e6,
                    "label": (40.8 + 3 * 18.4 + 17.8) * 1e6},
    "blobs_1m_d2": {"source": "609bf7a7ba72f254", "ringk": 121.5e6, "search": (128.2 + 1.4) * 1e6,
                    "density": 67.5e6, "finish": 194.6e6, "peaks": (43.8 + 93.5) * 1e6,
                    "label": (53.0 + 3 * 40.5 + 39.1) * 1e6},
}


def source_hash(files) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_traffic(group: str, workload: str):
    rec = HBM_BYTES.get(workload)
    if rec is None or rec.get("source") != source_hash(KERNEL_SOURCES):
        return None
    return rec.get(group)


def cpu_baseline(job, budget_s: float) -> dict:
    """The C oracle (plain O(n^2) scan) on a uniform subsample of the workload.

    Its cost grows as n^2 (every point scans all points for rho, and its density
    prefix for the dependent point), so points/s at the full size is the
    sample's points/s times m/n.  The sample size m is grown until one run
    takes a good part of `budget_s`.
    """
    import numpy as np

    from oracle import scan

    rng = np.random.default_rng(99)
    m = 4000
    elapsed = 0.0
    while True:
        idx = np.sort(rng.choice(job.n, size=min(m, job.n), replace=False))
        sub = np.ascontiguousarray(job.pts[idx])
        t0 = time.perf_counter()
        scan.dpc(sub, job.d_cut, job.rho_min, job.delta_min)
        elapsed = time.perf_counter() - t0
        if elapsed > budget_s / 4 or m >= job.n:
            break
        m = int(min(job.n, m * max(1.5, min(4.0, math.sqrt(budget_s / 2.5 / max(elapsed, 1e-3))))))
    pps_sample = m / elapsed
    value = pps_sample * m / job.n if m < job.n else pps_sample
    return {"value": value, "unit": "points/s", "cores": scan.threads(), "kind": "oracle",
            "sample": f"full oracle (rho, dependent, labels) on a uniform random subsample of {m} of the "
                      f"{job.n} points ({elapsed:.2f} s); points/s scaled by m/n since its cost is O(n^2)"}


def _make_job(spec):
    return spec.make()


def make_batch_jobs(count: int):
    """The batch workload's jobs, drawn in a process pool (before any GPU use)."""
    import concurrent.futures as cf

    from paper_2207_04649_amd import inputs

    specs = inputs.batch_specs(count)
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(workers) as ex:
        return list(ex.map(_make_job, specs, chunksize=16))


def make_serve_requests(duration: float):
    """Requests of the served workload's trace; new jobs drawn in a process pool (before any GPU use)."""
    import concurrent.futures as cf

    from paper_2207_04649_amd import inputs, serve

    trace = inputs.serve_trace(duration=duration)
    specs = [r.spec for r in trace if r.kind == "new"]
    workers = max(1, min(16, os.cpu_count() or 1))
    jobs = {}
    with cf.ProcessPoolExecutor(workers) as ex:
        for k, (sp, job) in enumerate(zip(specs, ex.map(_make_job, specs, chunksize=4))):
            jobs[sp.seed] = job
            if (k + 1) % 1000 == 0:
                print(f"serve: {k + 1} of {len(specs)} new jobs drawn", file=sys.stderr, flush=True)
    return serve.trace_requests(trace, lambda spec: jobs[spec.seed])


def bench_serve(args, reqs) -> int:
    """Replay the Poisson trace in real time through the continuous-batching
    server; the same trace through one slot without grouping for comparison."""
    import copy

    import torch

    from paper_2207_04649_amd import dpc, inputs, serve

    warm = inputs.blob_job(1, 5000, 3, 5, 500.0, 4000.0, 0.05)  # module load and first launches
    t = torch.from_numpy(warm.pts).cuda()
    dpc.dpc_run(t, warm.d_cut, warm.rho_min, warm.delta_min)
    torch.cuda.synchronize()
    results = {}
    # continuous: `slots` streams for new jobs (small ones grouped) and one of its own for
    # re-thresholds; the comparison: one stream, every request in arrival order
    for name, slots, group, relabel in (("continuous", args.slots, True, 8), ("one_slot_fifo", 1, False, 0)):
        rq = [copy.copy(q) for q in reqs]
        srv = serve.Server(budget_bytes=64 << 30, slots=slots, group_small=group, relabel_slots=relabel)
        t0 = time.perf_counter()
        def progress(k, n, name=name, srv=srv, t0=t0):
            staged = sum(b.numel() for b in srv.stage_in + srv.stage_out if b is not None)
            with open("/proc/self/statm") as f:
                rss = int(f.read().split()[1]) * os.sysconf("SC_PAGE_SIZE")
            print(f"{name}: {k} of {n} requests done, {time.perf_counter() - t0:.1f} s, pinned staging "
                  f"{staged / 2 ** 20:.0f} MiB, host RSS {rss / 2 ** 30:.2f} GiB", file=sys.stderr, flush=True)

        srv.run(rq, progress=progress)
        wall = time.perf_counter() - t0
        done = [q for q in rq if not q.dropped]
        results[name] = {"latency": serve.latency_summary(rq), "wall_s": wall,
                         "requests_per_s": len(done) / wall,
                         "new_points_per_s": sum(q.pts.shape[0] for q in done if q.kind == "new") / wall,
                         "stats": dict(srv.stats), "peak_hbm_gb": srv.peak_used / 2 ** 30}
        print(f"{name}: {json.dumps(results[name])}", file=sys.stderr, flush=True)
    main_r = results["continuous"]
    line = {
        "metric": "served DPC latency, arrival -> labels in pinned host memory (p99 of new jobs), 1 MI355X",
        "value": main_r["latency"]["new"]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": main_r["wall_s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serve", "duration_s": args.duration, "rate_per_s": 200.0,
                   "requests": len(reqs), "new": sum(1 for q in reqs if q.kind == "new"),
                   "rethreshold": sum(1 for q in reqs if q.kind == "rethreshold"), "slots": args.slots,
                   "relabel_slots": 8, "hbm_budget_gb": 64},
        "latency": main_r["latency"],
        "requests_per_s": main_r["requests_per_s"],
        "new_points_per_s": main_r["new_points_per_s"],
        "stats": main_r["stats"],
        "peak_hbm_gb": main_r["peak_hbm_gb"],
        "one_slot_fifo": {"latency": results["one_slot_fifo"]["latency"],
                          "requests_per_s": results["one_slot_fifo"]["requests_per_s"]},
    }
    print(json.dumps(line), flush=True)
    return 0


def bench_batch(args, jobs) -> int:
    """Many-job batch: all jobs through dpc_batch_run (one launch per phase and
    dimension), against the same jobs launched one dpc_run at a time."""
    import torch

    from paper_2207_04649_amd import autotune, dpc

    dev = torch.device("cuda:0")
    problems = [(torch.from_numpy(j.pts).to(dev), j.d_cut, j.rho_min, j.delta_min) for j in jobs]
    total = sum(j.n for j in jobs)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    table = {} if args.no_autotune else autotune.tune(problems, log=log)
    tun = autotune.tunings_for(problems, table) if table else None
    b = dpc.Batch(problems, tun)
    for _ in range(max(1, args.warmup)):
        b.run()
    b.sync_status()

    L = dpc.lib()
    L.dpc_profile_enable.argtypes = [ctypes.c_int32]
    L.dpc_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    buf = ctypes.create_string_buffer(8192)
    L.dpc_profile_report(buf, 8192)
    L.dpc_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.dpc_profile_enable(0)
    L.dpc_profile_report(buf, 8192)
    prof = json.loads(buf.value.decode())
    b.sync_status()
    batched_s = (t1 - t0) / args.steps

    # The same batch replayed from a captured HIP graph.
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            dpc.dpc_batch_run(b.handle, b.ws, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / args.steps
    b.sync_status()

    # One dpc_run launch sequence per job, workspaces allocated beforehand.
    wss = [dpc.workspace(j.n, j.d, j.d_cut, dev) for j in jobs]
    outs = [{} for _ in jobs]
    for (pt, dc, rm, dm), ws, o in zip(problems, wss, outs):
        dpc.dpc_run(pt, dc, rm, dm, ws=ws, out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (pt, dc, rm, dm), ws, o in zip(problems, wss, outs):
        dpc.dpc_run(pt, dc, rm, dm, ws=ws, out=o)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t0
    same = all(torch.equal(b.out[k][f], outs[k][f]) for k in range(0, len(jobs), max(1, len(jobs) // 256))
               for f in ("rho", "dep", "delta", "label", "ncenters"))

    sum_ops = sum(int(o["rho"].sum().item()) * test_ops(j.d) for o, j in zip(b.out, jobs))
    dens_ms = prof["density"][1] / max(1, prof["density"][0])
    achieved = sum_ops / (dens_ms * 1e-3) / 1e12
    line = {
        "metric": "points/s batched DPC (rho+delta+labels), 4096 jobs per launch sequence, 1 MI355X",
        "value": total / batched_s,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": batched_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batch4096", "jobs": len(jobs), "points": total,
                   "dims": sorted({j.d for j in jobs}), "n_range": [min(j.n for j in jobs), max(j.n for j in jobs)]},
        "graph_replay": {"value": total / graph_s, "ms_per_step": graph_s * 1e3},
        "per_job_launches": {"value": total / single_s, "ms_per_step": single_s * 1e3},
        "batched_vs_per_job": single_s / batched_s,
        "batch_equals_per_job": same,
        "autotune": {f"d{k[0]}_size{k[1]}": v["options"] for k, v in table.items()},
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in prof.items() if k != "work" and v[0]},
        "roofline": {"kernel": "density", "avg_ms": dens_ms, "bound": "alu", "achieved": achieved,
                     "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None},
    }
    print(json.dumps(line), flush=True)
    b.close()
    return 0 if same else 1


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="walks_4m_d4")
    ap.add_argument("--extra", default="blobs_1m_d2", help="a second workload measured as an extra key ('' for none)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-approx", action="store_true", help="skip the Approx-DPC lines")
    ap.add_argument("--approx-only", action="store_true", help="time Approx-DPC alone on --workload")
    ap.add_argument("--sapprox-only", action="store_true", help="time S-Approx-DPC alone on --workload")
    ap.add_argument("--eps", type=float, default=0.5, help="S-Approx-DPC's eps")
    ap.add_argument("--jobs", type=int, default=4096, help="jobs of the batch4096 workload")
    ap.add_argument("--no-autotune", action="store_true", help="batch4096: library defaults for every job")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of the Poisson trace")
    ap.add_argument("--slots", type=int, default=4, help="serve: concurrent slots (streams)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy kernel of known size, "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU sharding is a design "
                                   "note, not an implementation", "n_gpus": args.gpus}))
        return 2

    batch_jobs = make_batch_jobs(args.jobs) if args.workload == "batch4096" else None
    serve_reqs = make_serve_requests(args.duration) if args.workload == "serve" else None

    import torch

    from paper_2207_04649_amd import dpc, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        return 1
    if batch_jobs is not None:
        return bench_batch(args, batch_jobs)
    if serve_reqs is not None:
        return bench_serve(args, serve_reqs)
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    job = inputs.WORKLOADS[args.workload]()
    if args.approx_only:  # Approx-DPC alone (for its kernel traces): no exact run, no comparison
        r = bench_approx(job, args.steps, args.warmup, None)
        print(json.dumps({"metric": "points/s end-to-end Approx-DPC (rho+delta+labels) at 1 MI355X",
                          "value": r["value"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": job.name, "n": job.n, "d": job.d, "d_cut": job.d_cut},
                          "kernels_ms_per_step": r["kernels_ms_per_step"],
                          "approximate_fraction": r["approximate_fraction"]}), flush=True)
        return 0
    if args.sapprox_only:  # S-Approx-DPC alone (for its kernel traces)
        r = bench_sapprox(job, args.steps, args.warmup, args.eps)
        print(json.dumps({"metric": "points/s end-to-end S-Approx-DPC (rho+delta+labels) at 1 MI355X",
                          "value": r["value"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
                          "config": {"workload": job.name, "n": job.n, "d": job.d, "d_cut": job.d_cut,
                                     "eps": args.eps},
                          "kernels_ms_per_step": r["kernels_ms_per_step"],
                          "picked_fraction": r["picked_fraction"]}), flush=True)
        return 0
    res = bench_single(args, job, args.steps, args.warmup, with_roofline=True)
    line = {
        "metric": "points/s end-to-end DPC (rho+delta+labels) at 1 MI355X",
        "value": res["value"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": job.name, "n": job.n, "d": job.d, "d_cut": job.d_cut, "rho_min": job.rho_min,
                   "delta_min": job.delta_min},
        "kernels_ms_per_step": res["kernels_ms_per_step"],
        "roofline": res["roofline"],
        "rooflines": res["rooflines"],
        "work": res["work"],
        "ncenters": res["ncenters"],
        "decision_graph": res["decision_graph"],
    }
    approx, sapprox = {}, {}
    if not args.no_approx:
        approx[job.name] = bench_approx(job, max(3, args.steps // 2), 2, res["label"])
        sapprox[job.name] = bench_sapprox(job, max(3, args.steps // 2), 2, args.eps, res["label"])
    if args.extra and args.extra != job.name:
        ex = inputs.WORKLOADS[args.extra]()
        r2 = bench_single(args, ex, max(3, args.steps // 2), 2, with_roofline=True)
        line["extra"] = {ex.name: {"value": r2["value"], "unit": "points/s", "ms_per_step": r2["ms_per_step"],
                                   "kernels_ms_per_step": r2["kernels_ms_per_step"],
                                   "roofline": r2["roofline"]}}
        if not args.no_approx:
            approx[ex.name] = bench_approx(ex, max(3, args.steps // 2), 2, r2["label"])
            sapprox[ex.name] = bench_sapprox(ex, max(3, args.steps // 2), 2, args.eps, r2["label"])
            # the time / accuracy trade-off over eps (the shape of Table 5)
            sapprox[ex.name]["eps_sweep"] = {
                str(e): {k: r[k] for k in ("ms_per_step", "picked_fraction", "rand_index_vs_exact")}
                for e in (0.25, 0.5, 1.0)
                for r in [bench_sapprox(ex, max(3, args.steps // 2), 1, e, r2["label"])]}
    if approx:
        line["approx_dpc"] = approx
        line["s_approx_dpc"] = sapprox
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(job, args.cpu_budget)
    print(json.dumps(line), flush=True)
    return 0


def _profile_lib():
    from paper_2207_04649_amd import dpc

    L = dpc.lib()
    L.dpc_profile_enable.argtypes = [ctypes.c_int32]
    L.dpc_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    L.dpc_profile_report.restype = ctypes.c_int32
    return L


def _report(L) -> dict:
    buf = ctypes.create_string_buffer(8192)
    L.dpc_profile_report(buf, 8192)
    return json.loads(buf.value.decode())


def bench_decision(job, out: dict, reps: int = 20) -> dict:
    """Decision-graph summaries (Section 2.1) of one run's resident rho and delta: top-100
    by delta, a 16 x 16 <rho, delta> histogram and the suggested delta_min, timed with
    HIP events over `reps` repetitions each."""
    import torch

    from paper_2207_04649_amd import dpc

    dev = out["rho"].device
    ws = torch.empty(dpc.DECISION_WS_BYTES, dtype=torch.uint8, device=dev)
    re = torch.logspace(0, 4, 17, dtype=torch.float64, device=dev)
    de = torch.cat([torch.zeros(1, dtype=torch.float64, device=dev),
                    torch.logspace(math.log10(job.d_cut / 8), math.log10(job.d_cut * 1e3), 15, dtype=torch.float64,
                                   device=dev), torch.tensor([math.inf], dtype=torch.float64, device=dev)])
    res = {}
    for name, fn in (("top100_ms", lambda: dpc.dpc_decision_top(out["rho"], out["delta"], job.rho_min, 100, ws=ws)),
                     ("histogram_16x16_ms", lambda: dpc.dpc_decision_histogram(out["rho"], out["delta"], re, de))):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        res[name] = a.elapsed_time(b) / reps
        if name == "top100_ms":
            top = r
    dmin, cent = dpc.dpc_decision_suggest(top, job.d_cut)
    res["suggested_delta_min"] = float(dmin.item())
    res["suggested_centers"] = int(cent.item())
    return res


def bench_single(args, job, steps: int, warmup: int, with_roofline: bool) -> dict:
    """Time `steps` dpc_run calls on resident input (HIP events per kernel group on the
    library's stream inside the timed region), then one untimed instrumented call for
    the kernels' candidate-test counts."""
    import torch

    from paper_2207_04649_amd import dpc

    dev = torch.device("cuda:0")
    pts = torch.from_numpy(job.pts).to(dev)
    ws = dpc.workspace(job.n, job.d, job.d_cut, dev)
    out: dict = {}
    for _ in range(warmup):
        dpc.dpc_run(pts, job.d_cut, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    dpc.dpc_sync_status(ws)

    L = _profile_lib()
    _report(L)  # clear
    L.dpc_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dpc.dpc_run(pts, job.d_cut, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.dpc_profile_enable(0)
    prof = _report(L)
    dpc.dpc_sync_status(ws)

    # one more call, untimed, counting each kernel's candidate tests
    L.dpc_profile_enable(2)
    dpc.dpc_run(pts, job.d_cut, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    L.dpc_profile_enable(0)
    work = _report(L)["work"]
    dpc.dpc_sync_status(ws)

    per = {k: v[1] / steps for k, v in prof.items() if k != "work" and v[0]}  # each group's ms per step
    sum_rho = int(out["rho"].sum().item())
    plan = dpc.dpc_plan(job.n, job.d, job.d_cut)
    roofs = rooflines(job, per, sum_rho, work, plan)
    dom = max((k for k in per if k in roofs), key=per.get)
    return {"value": job.n * steps / (t1 - t0), "ms_per_step": (t1 - t0) * 1000.0 / steps,
            "kernels_ms_per_step": {k: v[1] / steps for k, v in prof.items() if k != "work" and v[0]},
            "roofline": dict(roofs[dom], kernel=dom), "rooflines": roofs,
            "work": dict(work, sum_rho=sum_rho), "ncenters": int(out["ncenters"].item()),
            "label": out["label"], "decision_graph": bench_decision(job, out)}


def rand_index(a, b) -> float:
    """Rand index of two device labelings (noise, -1, counts as one more cluster): the
    fraction of point pairs on which they agree, from the contingency counts."""
    import torch

    ia = torch.unique(a, return_inverse=True)[1].to(torch.int64)
    ib = torch.unique(b, return_inverse=True)[1].to(torch.int64)
    pair = torch.unique(ia * (int(ib.max().item()) + 1) + ib, return_counts=True)[1]

    def c2(x):
        x = x.to(torch.int64)
        return int((x * (x - 1) // 2).sum().item())

    n = a.numel()
    tot = n * (n - 1) // 2
    return (tot + 2 * c2(pair) - c2(torch.bincount(ia)) - c2(torch.bincount(ib))) / tot


def bench_sapprox(job, steps: int, warmup: int, eps: float, exact_label=None) -> dict:
    """Time `steps` dpc_sapprox_run calls (S-Approx-DPC, Section 5) on resident input; with
    the exact labels, also their Rand index against S-Approx-DPC's."""
    import torch

    from paper_2207_04649_amd import dpc

    dev = torch.device("cuda:0")
    pts = torch.from_numpy(job.pts).to(dev)
    ws = torch.empty(dpc.dpc_sapprox_workspace_bytes(job.n, job.d, job.d_cut, eps), dtype=torch.uint8, device=dev)
    out: dict = {}
    for _ in range(warmup):
        dpc.dpc_sapprox_run(pts, job.d_cut, eps, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    dpc.dpc_sync_status(ws)
    L = _profile_lib()
    _report(L)
    L.dpc_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dpc.dpc_sapprox_run(pts, job.d_cut, eps, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.dpc_profile_enable(0)
    prof = _report(L)
    dpc.dpc_sync_status(ws)
    return {"eps": eps, "value": job.n * steps / (t1 - t0), "unit": "points/s",
            "ms_per_step": (t1 - t0) * 1000.0 / steps,
            "kernels_ms_per_step": {k: v[1] / steps for k, v in prof.items() if k != "work" and v[0]},
            "picked_fraction": float(out["picked"].float().mean().item()),
            "ncenters": int(out["ncenters"].item()),
            "rand_index_vs_exact": None if exact_label is None else rand_index(out["label"], exact_label)}


def bench_approx(job, steps: int, warmup: int, exact_label) -> dict:
    """Time `steps` dpc_approx_run calls (Approx-DPC, Section 4) on resident input, with
    HIP events per kernel group; report how many points the approximation rules settled
    and whether the centers equal the exact path's (`exact_label`, a device tensor)."""
    import torch

    from paper_2207_04649_amd import dpc

    dev = torch.device("cuda:0")
    pts = torch.from_numpy(job.pts).to(dev)
    ws = torch.empty(dpc.dpc_approx_workspace_bytes(job.n, job.d, job.d_cut), dtype=torch.uint8, device=dev)
    out: dict = {}
    for _ in range(warmup):
        dpc.dpc_approx_run(pts, job.d_cut, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    dpc.dpc_sync_status(ws)
    L = _profile_lib()
    _report(L)
    L.dpc_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dpc.dpc_approx_run(pts, job.d_cut, job.rho_min, job.delta_min, ws=ws, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.dpc_profile_enable(0)
    prof = _report(L)
    dpc.dpc_sync_status(ws)
    same = None
    if exact_label is not None:
        ids = torch.arange(job.n, device=dev, dtype=torch.int32)
        same = bool(torch.equal(out["label"] == ids, exact_label == ids)) and bool(
            torch.equal(out["label"] < 0, exact_label < 0))
    return {"value": job.n * steps / (t1 - t0), "unit": "points/s", "ms_per_step": (t1 - t0) * 1000.0 / steps,
            "kernels_ms_per_step": {k: v[1] / steps for k, v in prof.items() if k != "work" and v[0]},
            "approximate_fraction": float(out["approx"].float().mean().item()),
            "centers_and_noise_equal_exact": same,
            "rand_index_vs_exact": None if exact_label is None else rand_index(out["label"], exact_label)}


if __name__ == "__main__":
    sys.exit(main())
