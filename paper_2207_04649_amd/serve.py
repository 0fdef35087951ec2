"""Served density-peaks clustering: continuous batching of new-job and
re-threshold requests on one GPU.

A request is either a new job (points, d_cut, rho_min, delta_min) or a
re-threshold of a resident job (new rho_min, delta_min).  The paper picks the
thresholds on the decision graph once rho and delta are known (Section 2.1), so
a resident job keeps its coordinates, rho, dep and delta in HBM and a
re-threshold reruns only the labelling (dpc_label, Defs. 4-6).

Scheduling.  Work runs in slots, one HIP stream each (default priority).  New
jobs and re-thresholds wait in two queues with slots of their own, so an O(n)
relabel never waits behind a new job's clustering: the loop admits arrived
requests of each queue in arrival order whenever one of its slots is free (and,
for a new job, when it fits the HBM budget).  Small new jobs that are waiting
together share one slot as a many-job batch (dpc_batch_run); a large one takes
a slot alone (dpc_run).  Idle resident jobs are evicted, least recently used
first, when a new job needs their memory.  Requests that arrive while others
are on the GPU are admitted as soon as a slot and memory free up, so their work
overlaps on the device.  Latency is arrival -> labels in pinned host memory.

Host staging.  Each slot owns two pinned host buffers, reused from request to
request: coordinates are copied into one and sent to the device from there,
labels (and, with keep_outputs, rho, dep and delta) come back into the other and
are copied out to the request when its work has ended.  Pinned memory therefore
stays bounded by the slots and the largest group, whatever the length of the
trace (pinning memory per request grows with the trace, and pinning tens of GB
can stall in the driver).

Every result equals that of the job run alone: the kernels are deterministic
and jobs share no device memory.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import dpc

SMALL_JOB = 65_536  # new jobs up to this size may share a slot as one batch
MAX_GROUP = 64      # most jobs per shared-slot batch


@dataclasses.dataclass(eq=False)
class Req:
    rid: int
    t_arrival: float            # seconds from the start of the run
    kind: str                   # "new" or "rethreshold"
    pts: np.ndarray | None = None
    d_cut: float = 0.0
    rho_min: int = 0
    delta_min: float = 0.0
    seed: int = -1              # new job: the seed of its generator spec
    pick: float = 0.0           # re-threshold: picks a ready resident job at admission
    delta_factor: float = 0.0   # re-threshold: delta_min = delta_factor * the job's d_cut
    job_key: int = -1           # the job the request created or re-thresholded
    t_done: float = -1.0
    dropped: bool = False       # re-threshold with no job ready (nothing to re-threshold)
    labels: torch.Tensor | None = None    # host copies (through the slot's pinned staging)
    ncenters: torch.Tensor | None = None
    rho: torch.Tensor | None = None       # new jobs, with keep_outputs: host copies
    dep: torch.Tensor | None = None
    delta: torch.Tensor | None = None


@dataclasses.dataclass(eq=False)
class Resident:
    key: int
    n: int
    d: int
    d_cut: float
    pts: torch.Tensor
    rho: torch.Tensor
    dep: torch.Tensor
    delta: torch.Tensor
    label: torch.Tensor
    ncenters: torch.Tensor
    bytes: int
    ready: bool = False         # rho, dep and delta computed
    busy: int = 0               # requests in flight that read it
    last_use: float = 0.0


@dataclasses.dataclass(eq=False)
class Inflight:
    event: torch.cuda.Event
    slot: int
    reqs: list
    jobs: list                  # Resident entries the work reads or writes
    ws_bytes: int               # workspace charged to the ledger until retirement
    keep: list                  # tensors and host buffers that must live until the work ends
    new: bool
    batch: object = None        # dpc_batch handle to free
    outs: list = dataclasses.field(default_factory=list)  # (request, field, staged host view)


class Server:
    """``slots`` streams for new jobs, ``relabel_slots`` for re-thresholds (0: they
    share the new-job slots and queue, one FIFO for both).  With ``keep_outputs``
    a new job's rho, dep and delta are copied to pinned host memory as well."""

    def __init__(self, budget_bytes: int = 64 << 30, slots: int = 4, device: str = "cuda:0",
                 group_small: bool = True, relabel_slots: int = 1, keep_outputs: bool = False):
        self.dev = torch.device(device)
        self.budget = int(budget_bytes)
        self.used = 0
        self.group_small = group_small
        self.keep_outputs = keep_outputs
        self.shared = relabel_slots <= 0
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots + max(0, relabel_slots))]
        self.free_slots = list(range(slots))                           # new jobs (and shared relabels)
        self.free_relabel = list(range(slots, slots + max(0, relabel_slots)))
        self.inflight: list[Inflight] = []
        self.resident: "collections.OrderedDict[int, Resident]" = collections.OrderedDict()
        self.next_key = 0
        self.label_ws = [torch.empty(dpc.DPC_LABEL_WS_BYTES, dtype=torch.uint8, device=self.dev)
                         for _ in range(len(self.streams))]
        self.stage_in: list = [None] * len(self.streams)   # pinned host staging per slot
        self.stage_out: list = [None] * len(self.streams)
        self.stats = collections.Counter()
        self.peak_used = 0
        self.new_outstanding = 0  # new-job requests of the run not yet admitted

    # ---- memory ledger ----
    @staticmethod
    def resident_bytes(n: int, d: int) -> int:
        return 4 * d * n + 16 * n + 4 * n + 8  # coordinates, rho/dep/delta, labels, ncenters

    def _make_room(self, need: int) -> bool:
        for key in list(self.resident.keys()):
            if self.used + need <= self.budget:
                break
            r = self.resident[key]
            if r.busy or not r.ready:
                continue
            del self.resident[key]
            self.used -= r.bytes
            self.stats["evicted"] += 1
        return self.used + need <= self.budget

    # ---- host staging ----
    @staticmethod
    def _stage(bufs: list, slot: int, nbytes: int) -> torch.Tensor:
        """The slot's pinned buffer of at least nbytes (grown at least twofold, never
        shrunk, so a slot allocates a few times at most; the slot's previous work has
        ended, so the old buffer is free)."""
        old = bufs[slot]
        if old is None or old.numel() < nbytes:
            grow = 2 * old.numel() if old is not None else 0
            bufs[slot] = torch.empty(max(nbytes, grow, 1 << 20), dtype=torch.uint8, pin_memory=True)
        return bufs[slot]

    @staticmethod
    def _carve(stage: torch.Tensor, at: int, count: int, dtype: torch.dtype) -> tuple[torch.Tensor, int]:
        """A view of `count` items of dtype at byte offset `at` (256-aligned); the next offset."""
        size = torch.empty(0, dtype=dtype).element_size() * count
        view = stage[at: at + size].view(dtype)
        return view, at + (size + 255) // 256 * 256

    def _out_views(self, reqs: list[Req], ns: list[int], slot: int, full: bool) -> list:
        """Staged host views of each request's outputs: [(req, {field: view})]."""
        per = [4 * n + 8 + (16 * n if full else 0) + 5 * 256 for n in ns]
        stage = self._stage(self.stage_out, slot, sum(per))
        at, views = 0, []
        for q, n in zip(reqs, ns):
            v = {}
            v["labels"], at = self._carve(stage, at, n, torch.int32)
            v["ncenters"], at = self._carve(stage, at, 1, torch.int64)
            if full:
                v["rho"], at = self._carve(stage, at, n, torch.int32)
                v["dep"], at = self._carve(stage, at, n, torch.int32)
                v["delta"], at = self._carve(stage, at, n, torch.float64)
            views.append((q, v))
        return views

    # ---- launching ----
    def _launch_new(self, reqs: list[Req], slot: int, now: float, ws_bytes: int) -> None:
        stream = self.streams[slot]
        jobs, keep = [], []
        batch = None
        stage = self._stage(self.stage_in, slot, sum(q.pts.nbytes + 256 for q in reqs))
        at = 0
        with torch.cuda.stream(stream):
            for q in reqs:
                n, d = q.pts.shape
                host, at = self._carve(stage, at, n * d, torch.int32)
                host.numpy()[:] = q.pts.reshape(-1)
                host = host.view(n, d)
                pts = host.to(self.dev, non_blocking=True)
                dev = lambda dt: torch.empty(n, dtype=dt, device=self.dev)  # noqa: E731
                r = Resident(q.job_key, n, d, q.d_cut, pts, dev(torch.int32), dev(torch.int32), dev(torch.float64),
                             dev(torch.int32), torch.empty(1, dtype=torch.int64, device=self.dev),
                             self.resident_bytes(n, d), busy=1, last_use=now)
                jobs.append(r)
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.dev)
            keep.append(ws)
            if len(reqs) == 1:
                q, r = reqs[0], jobs[0]
                out = {"rho": r.rho, "dep": r.dep, "delta": r.delta, "label": r.label, "ncenters": r.ncenters}
                dpc.dpc_run(r.pts, r.d_cut, q.rho_min, q.delta_min, ws=ws, out=out, stream=stream)
            else:
                js = [dpc.Job(r.pts.data_ptr(), r.n, r.d, r.d_cut, q.rho_min, q.delta_min, r.rho.data_ptr(),
                              r.dep.data_ptr(), r.delta.data_ptr(), r.label.data_ptr(), r.ncenters.data_ptr())
                      for q, r in zip(reqs, jobs)]
                batch, nbytes = dpc.dpc_batch_plan(js)
                assert nbytes <= ws_bytes
                dpc.dpc_batch_bind(batch, ws)
                dpc.dpc_batch_run(batch, ws, stream=stream)
            outs = self._out_views(reqs, [r.n for r in jobs], slot, self.keep_outputs)
            for (q, v), r in zip(outs, jobs):
                v["labels"].copy_(r.label, non_blocking=True)
                v["ncenters"].copy_(r.ncenters, non_blocking=True)
                if self.keep_outputs:
                    v["rho"].copy_(r.rho, non_blocking=True)
                    v["dep"].copy_(r.dep, non_blocking=True)
                    v["delta"].copy_(r.delta, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        for r in jobs:
            self.resident[r.key] = r
        self.inflight.append(Inflight(ev, slot, reqs, jobs, ws_bytes, keep, True, batch, outs))
        self.stats["new_launches"] += 1
        self.stats["new_jobs"] += len(reqs)

    def _launch_relabel(self, q: Req, r: Resident, slot: int, now: float) -> None:
        stream = self.streams[slot]
        r.busy += 1
        r.last_use = now
        self.resident.move_to_end(r.key)
        with torch.cuda.stream(stream):
            lab = torch.empty(r.n, dtype=torch.int32, device=self.dev)
            nc = torch.empty(1, dtype=torch.int64, device=self.dev)
            dpc.dpc_label(r.rho, r.dep, r.delta, q.rho_min, q.delta_min, label=lab, ncenters=nc,
                          ws=self.label_ws[slot], stream=stream)
            outs = self._out_views([q], [r.n], slot, False)
            outs[0][1]["labels"].copy_(lab, non_blocking=True)
            outs[0][1]["ncenters"].copy_(nc, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight.append(Inflight(ev, slot, [q], [r], 0, [lab, nc], False, None, outs))
        self.stats["relabels"] += 1

    def _retire(self, now: float) -> int:
        done, keep = 0, []
        for f in self.inflight:
            if not f.event.query():
                keep.append(f)
                continue
            for q in f.reqs:
                q.t_done = now
            for q, v in f.outs:  # out of the slot's staging buffer before the slot is reused
                for field, view in v.items():
                    setattr(q, field, view.clone())
            for r in f.jobs:
                r.busy -= 1
                if f.new:
                    r.ready = True
            self.used -= f.ws_bytes
            if f.batch is not None:
                dpc.dpc_batch_free(f.batch)
            (self.free_slots if f.new or self.shared else self.free_relabel).append(f.slot)
            done += len(f.reqs)
        self.inflight = keep
        return done

    @staticmethod
    def _group_ws_bytes(group: list[Req]) -> int:
        if len(group) == 1:
            n, d = group[0].pts.shape
            return dpc.dpc_workspace_bytes(n, d, group[0].d_cut)
        fake = [dpc.Job(4096, g.pts.shape[0], g.pts.shape[1], g.d_cut, g.rho_min, g.delta_min,
                        4096, 4096, 4096, 4096, 4096) for g in group]
        h, nbytes = dpc.dpc_batch_plan(fake)
        dpc.dpc_batch_free(h)
        return nbytes

    def _admit(self, queue: "collections.deque[Req]", now: float) -> bool:
        """Launch the head of the queue if a slot and memory allow; False if it must wait."""
        q = queue[0]
        if q.kind == "rethreshold":
            ready = [k for k, r in self.resident.items() if r.ready]
            if not ready:
                # Wait for a job being computed, or (with a queue of its own) for one
                # still to come.  With one queue for everything a job still to come is
                # behind this request, so waiting for it would stall the queue for good.
                if any(not r.ready for r in self.resident.values()) or (self.new_outstanding and not self.shared):
                    return False
                queue.popleft()
                q.dropped = True
                q.t_done = now
                self.stats["dropped"] += 1
                return True
            r = self.resident[ready[min(int(q.pick * len(ready)), len(ready) - 1)]]
            q.job_key = r.key
            q.delta_min = q.delta_factor * r.d_cut
            queue.popleft()
            self._launch_relabel(q, r, (self.free_slots if self.shared else self.free_relabel).pop(0), now)
            return True
        group = [q]
        if self.group_small and q.pts.shape[0] <= SMALL_JOB:
            for other in list(queue)[1:]:
                if len(group) >= MAX_GROUP:
                    break
                if other.kind == "new" and other.pts.shape[0] <= SMALL_JOB:
                    group.append(other)
        while True:  # the largest leading part of the group that fits (after evictions)
            ws_bytes = self._group_ws_bytes(group)
            need = ws_bytes + sum(self.resident_bytes(*g.pts.shape) for g in group)
            if self.used + need <= self.budget or self._make_room(need):
                break
            if len(group) == 1:
                return False
            group = group[: len(group) // 2]
        for g in group:
            queue.remove(g)
            g.job_key = self.next_key
            self.next_key += 1
        self.new_outstanding -= len(group)
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        self._launch_new(group, self.free_slots.pop(0), now, ws_bytes)
        return True

    def run(self, requests: list[Req], clock=time.perf_counter, progress=None) -> list[Req]:
        """Replay `requests` in real time (by t_arrival); returns them with t_done set.
        ``progress(finished, total)`` is called each time another 1000 requests have
        finished, and at least every 20 s."""
        pending = collections.deque(sorted(requests, key=lambda q: q.t_arrival))
        queues = {"new": collections.deque(), "rethreshold": collections.deque()}
        self.new_outstanding = sum(1 for q in requests if q.kind == "new")
        finished = 0
        reported = 0
        t0 = clock()
        t_report = t0
        while finished < len(requests):
            if progress is not None and (finished >= reported + 1000 or clock() - t_report >= 20.0):
                reported = max(reported, finished - finished % 1000)
                t_report = clock()
                progress(finished, len(requests))
            now = clock() - t0
            while pending and pending[0].t_arrival <= now:
                q = pending.popleft()
                queues["new" if self.shared else q.kind].append(q)
            finished += self._retire(now)
            progressed = False
            for kind in ("rethreshold", "new"):
                queue = queues[kind]
                free = self.free_relabel if (kind == "rethreshold" and not self.shared) else self.free_slots
                # every waiting re-threshold a slot allows, but one new launch per pass:
                # a launch's host work (staging, planning) must not hold re-thresholds back
                budget = len(queue) if kind == "rethreshold" else 1
                while queue and free and budget > 0:
                    budget -= 1
                    dropped = self.stats["dropped"]
                    if not self._admit(queue, now):
                        if not self.inflight and queue[0].kind == "new":
                            raise RuntimeError("a job does not fit the HBM budget even with nothing resident")
                        break
                    progressed = True
                    finished += self.stats["dropped"] - dropped
            if not progressed:
                time.sleep(0.0002)
        torch.cuda.synchronize()
        return requests


def latency_summary(reqs: list[Req]) -> dict:
    out = {}
    for kind in ("new", "rethreshold"):
        lat = np.array([1e3 * (q.t_done - q.t_arrival) for q in reqs if q.kind == kind and not q.dropped],
                       dtype=np.float64)
        if lat.size:
            out[kind] = {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean())}
    return out


def trace_requests(trace, make_job) -> list[Req]:
    """Requests of an inputs.serve_trace: new jobs drawn with make_job(spec)."""
    reqs = []
    for k, r in enumerate(trace):
        if r.kind == "new":
            job = make_job(r.spec)
            reqs.append(Req(k, r.t, "new", pts=job.pts, d_cut=job.d_cut, rho_min=job.rho_min,
                            delta_min=job.delta_min, seed=r.spec.seed))
        else:
            reqs.append(Req(k, r.t, "rethreshold", rho_min=r.rho_min, pick=r.pick, delta_factor=r.delta_factor))
    return reqs
