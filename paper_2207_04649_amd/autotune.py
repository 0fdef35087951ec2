"""Autotuner for many-job batches: per dimension, the plan options (cell
subdivision, strip width, search stages) with the shortest measured batch time.

Candidates are timed with real batch launches (dpc_batch_run) on a sample of
the jobs of each dimension; every candidate gives the same results (the options
change only how the exact search is organised), so the choice is a pure timing
decision.
"""
from __future__ import annotations

import time

import torch

from . import dpc

# Options tried for every dimension; the first is the library's default.
CANDIDATES = [
    {},
    {"subdiv": 1},
    {"subdiv": 2},
    {"subdiv": 3},
    {"stages": [(1, 1)]},
    {"stages": [(1, 1), (2, 4)]},
    {"strip_cells": 16},
    {"subdiv": 2, "stages": [(1, 1)]},
    {"grid_dims": 2},
    {"grid_dims": 2, "subdiv": 4},
    {"grid_dims": 8},                      # every coordinate indexed
    {"grid_dims": 8, "stages": [(1, 1)]},
]


def _time_batch(problems, tuning, reps: int) -> float:
    b = dpc.Batch(problems, [tuning] * len(problems))
    try:
        b.run()
        b.sync_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    finally:
        b.close()


def tune(problems, sample: int = 48, reps: int = 3, log=None) -> dict:
    """problems: list of (pts tensor, d_cut, rho_min, delta_min).  Returns
    {d: {"options": dict, "ms": {candidate index: ms}}} for every dimension present."""
    by_d: dict[int, list] = {}
    for pr in problems:
        by_d.setdefault(int(pr[0].shape[1]), []).append(pr)
    out = {}
    for d, prs in sorted(by_d.items()):
        step = max(1, len(prs) // sample)
        smp = prs[::step][:sample]
        times = {}
        for ci, opt in enumerate(CANDIDATES):
            times[ci] = 1e3 * _time_batch(smp, dpc.Tuning.make(**opt), reps)
        best = min(times, key=times.get)
        out[d] = {"options": CANDIDATES[best], "ms": times}
        if log:
            log(f"autotune d={d}: {len(smp)} sample jobs, best {CANDIDATES[best]} "
                f"({times[best]:.3f} ms vs default {times[0]:.3f} ms)")
    return out


def tunings_for(problems, table: dict) -> list:
    return [dpc.Tuning.make(**table[int(pr[0].shape[1])]["options"]) for pr in problems]
