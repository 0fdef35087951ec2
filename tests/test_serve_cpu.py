"""Host logic of the serving loop that needs no GPU.

* A re-threshold at the head of the one shared queue, with no job computed or
  being computed, must not wait for a job that can only arrive behind it (that
  wait never ends).
* The whole loop on a simulated device (events that complete after a delay):
  every request finishes, in both modes and under an evicting budget, and the
  HBM ledger ends charged with exactly the resident jobs."""
import collections
import time

import numpy as np
import pytest

from paper_2207_04649_amd import serve


def _server(shared: bool, outstanding: int):
    srv = object.__new__(serve.Server)  # the admission logic only, without streams
    srv.resident = {}
    srv.new_outstanding = outstanding
    srv.shared = shared
    srv.stats = collections.Counter()
    return srv


def _rethreshold():
    return serve.Req(rid=0, t_arrival=0.0, kind="rethreshold", rho_min=1, pick=0.5, delta_factor=2.0)


def test_shared_queue_drops_instead_of_waiting_for_a_job_behind_it():
    srv = _server(shared=True, outstanding=3)
    q = _rethreshold()
    queue = collections.deque([q])
    assert srv._admit(queue, 1.0) is True
    assert q.dropped and not queue and srv.stats["dropped"] == 1


def test_own_queue_waits_for_a_job_still_to_come():
    srv = _server(shared=False, outstanding=3)
    queue = collections.deque([_rethreshold()])
    assert srv._admit(queue, 1.0) is False and len(queue) == 1


def test_nothing_to_come_drops_in_both_modes():
    for shared in (True, False):
        srv = _server(shared=shared, outstanding=0)
        q = _rethreshold()
        assert srv._admit(collections.deque([q]), 1.0) is True and q.dropped


# ---------------------------------------------------------------- the whole loop, simulated

class _Done:
    """An event that completes at a given time of the simulation's clock."""

    def __init__(self, t_end: float):
        self.t_end = t_end

    def query(self) -> bool:
        return time.perf_counter() >= self.t_end


class _SimServer(serve.Server):
    """The serving loop's admission, grouping, eviction and retirement as they are,
    with the device work replaced by events that complete after n * 2 ns."""

    def __init__(self, slots, relabel_slots, budget, group_small=True):
        self.budget = budget
        self.used = 0
        self.group_small = group_small
        self.keep_outputs = False
        self.shared = relabel_slots <= 0
        self.free_slots = list(range(slots))
        self.free_relabel = list(range(slots, slots + max(0, relabel_slots)))
        self.inflight = []
        self.resident = collections.OrderedDict()
        self.next_key = 0
        self.stats = collections.Counter()
        self.peak_used = 0
        self.new_outstanding = 0

    @staticmethod
    def _group_ws_bytes(group):
        return sum(64 * g.pts.shape[0] for g in group)

    def _launch_new(self, reqs, slot, now, ws_bytes):
        jobs = []
        for q in reqs:
            n, d = q.pts.shape
            r = serve.Resident(q.job_key, n, d, q.d_cut, None, None, None, None, None, None,
                               self.resident_bytes(n, d), busy=1, last_use=now)
            jobs.append(r)
            self.resident[r.key] = r
        cost = 2e-9 * sum(q.pts.shape[0] for q in reqs)
        self.inflight.append(serve.Inflight(_Done(time.perf_counter() + cost), slot, reqs, jobs, ws_bytes, [], True))
        self.stats["new_launches"] += 1

    def _launch_relabel(self, q, r, slot, now):
        r.busy += 1
        r.last_use = now
        self.resident.move_to_end(r.key)
        self.inflight.append(serve.Inflight(_Done(time.perf_counter() + 1e-5), slot, [q], [r], 0, [], False))
        self.stats["relabels"] += 1


def _trace(seed, count, span):
    rng = np.random.default_rng(seed)
    reqs = []
    for i, t in enumerate(np.sort(rng.uniform(0.0, span, count))):
        if rng.random() < 0.3:
            reqs.append(serve.Req(i, float(t), "rethreshold", rho_min=1, pick=float(rng.random()),
                                  delta_factor=2.0))
        else:
            n = int(rng.choice([500, 5000, 50000, 400000]))
            reqs.append(serve.Req(i, float(t), "new", pts=np.zeros((n, 3), np.int32), d_cut=10.0, rho_min=1,
                                  delta_min=20.0))
    return reqs


@pytest.mark.parametrize("slots,relabel,budget_mb", [(4, 8, 1 << 14), (4, 2, 64), (1, 0, 1 << 14), (1, 0, 64)])
@pytest.mark.timeout(120)
def test_simulated_loop_finishes_every_request(monkeypatch, slots, relabel, budget_mb):
    # the loop ends with a device synchronisation: nothing to wait for here
    monkeypatch.setattr(serve.torch.cuda, "synchronize", lambda *a, **k: None)
    srv = _SimServer(slots, relabel, budget_mb << 20)
    reqs = _trace(7, 600, 0.3)
    peak = []
    srv.run(reqs, progress=lambda k, n: peak.append(srv.used))
    for q in reqs:
        assert q.t_done >= q.t_arrival, (q.rid, q.kind)
        assert q.kind == "rethreshold" or not q.dropped
    assert srv.peak_used <= srv.budget
    # every workspace is returned: what stays charged is exactly the resident jobs
    assert srv.used == sum(r.bytes for r in srv.resident.values())
    assert all(r.ready and r.busy == 0 for r in srv.resident.values())
    assert srv.stats["relabels"] + srv.stats["dropped"] == sum(q.kind == "rethreshold" for q in reqs)
    if budget_mb == 64:
        assert srv.stats["evicted"] > 0
