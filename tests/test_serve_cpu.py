"""Host logic of the serving loop that needs no GPU: a re-threshold at the head
of the one shared queue, with no job computed or being computed, must not wait
for a job that can only arrive behind it (that wait never ends)."""
import collections

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
