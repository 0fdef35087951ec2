"""Autotuner for many-job batches: per dimension and size class, the plan
options (kernel form, cell subdivision, strip width, search stages, ring cap)
with the shortest measured batch time.

Candidates are timed with real batch launches (dpc_batch_run) on a sample of
the jobs of each (dimension, size class); every candidate gives the same results
(the options change only how the exact search is organised), so the choice is a
pure timing decision.
"""
from __future__ import annotations

import time

import torch

from . import dpc

# Options tried for every class; the first is the library's default.
CANDIDATES = [
    {},
    {"lanes": 1},                          # 64-query tasks sharing windows
    {"lanes": 2},                          # one query per lane
    {"lanes": 2, "grid_dims": 8},          # one query per lane, every coordinate indexed
    {"lanes": 2, "stages": [(0, 1)]},      # one query per lane, the ball stage
    {"lanes": 2, "ring_cap": 384},
    {"lanes": 2, "open_radius": 2},        # one query per lane, a second lane stage for open points
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
    {"ring_cap": 24},
    {"ring_cap": 768},
]

# Size classes within a dimension: upper bounds on n (the last is open).
SIZE_CLASSES = (4_000, 16_000)


def size_class(n: int) -> int:
    for k, hi in enumerate(SIZE_CLASSES):
        if n < hi:
            return k
    return len(SIZE_CLASSES)


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


def _key(pr) -> tuple[int, int]:
    return int(pr[0].shape[1]), size_class(int(pr[0].shape[0]))


def tune(problems, sample: int = 48, reps: int = 3, log=None) -> dict:
    """problems: list of (pts tensor, d_cut, rho_min, delta_min).  Returns
    {(d, size class): {"options": dict, "ms": {candidate index: ms}}} for every class present."""
    by_key: dict[tuple, list] = {}
    for pr in problems:
        by_key.setdefault(_key(pr), []).append(pr)
    out = {}
    for key, prs in sorted(by_key.items()):
        step = max(1, len(prs) // sample)
        smp = prs[::step][:sample]
        times = {}
        for ci, opt in enumerate(CANDIDATES):
            times[ci] = 1e3 * _time_batch(smp, dpc.Tuning.make(**opt), reps)
        best = min(times, key=times.get)
        out[key] = {"options": CANDIDATES[best], "ms": times}
        if log:
            log(f"autotune d={key[0]} size class {key[1]}: {len(smp)} sample jobs, best {CANDIDATES[best]} "
                f"({times[best]:.3f} ms vs default {times[0]:.3f} ms)")
    return out


def tunings_for(problems, table: dict) -> list:
    return [dpc.Tuning.make(**table[_key(pr)]["options"]) for pr in problems]
