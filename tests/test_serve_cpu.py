"""Host logic of the request server, without a GPU: the sizing of a request,
the building of a slot and the solve are replaced by stand-ins, so what runs
is the admission, the slot pool and the failure handling alone."""
import numpy as np
import pytest

from paper_1009_0798_amd import _lib
from paper_1009_0798_amd import serve as S

FP = 10


def _request(rid, shape=1):
    """A request whose shape key is set by `shape` (base box width)."""
    return S.Request(rid=rid, arrival=0.0, base_blocks=(shape, 1, 1), dx0=0.125,
                     levels=[np.zeros((1, 3), np.int32)], B=[np.zeros((3, 1, 8, 8, 8))],
                     eta=[np.ones((1, 8, 8, 8))], dt=1.0)


class FakeSlot:
    def __init__(self, req):
        self.key = S.shape_key(req)
        self.bytes = FP
        self.closed = False
        self.last_used = 0.0

    def close(self):
        self.closed = True


def _stub(monkeypatch, srv, fail_solve=(), sizes=None, log=None):
    def footprint(req, opts):
        if sizes and req.rid in sizes:
            v = sizes[req.rid]
            if isinstance(v, Exception):
                raise v
            return v
        return FP

    made = []

    def make_slot(req, stream):
        s = FakeSlot(req)
        made.append(s)
        return s

    def solve(req, slot, stream):
        if log is not None:
            log.append((req.rid, id(slot), srv.resident))
        if req.rid in fail_solve:
            raise _lib.OhmError(_lib.OHM_ERR_NONFINITE, "eta is not finite")
        return 0, [dict(iters=1, mg_apps=1, rel_res=0.0, max_res=(0.0, 0.0, 0.0))], []

    monkeypatch.setattr(S, "footprint", footprint)
    monkeypatch.setattr(srv, "_make_slot", make_slot)
    monkeypatch.setattr(srv, "_solve", solve)
    srv.streams = [None] * srv.n_streams
    return made


@pytest.mark.timeout(60)
def test_failures_finish_their_requests_and_return_the_budget(monkeypatch):
    """Request 3 (a shape of its own) is refused at sizing, as the library
    refuses blocks outside the base grid; request 1 raises inside the solve.
    With a budget of one slot, a lost budget would starve every later request;
    instead all six finish, the two failures with their library status and
    message, the failed request's slot is closed, and the others reuse one
    resident slot, whose memory shutdown() returns."""
    srv = S.Server(hbm_budget=FP, n_streams=2)
    log = []
    made = _stub(monkeypatch, srv, fail_solve=(1,),
                 sizes={3: _lib.OhmError(_lib.OHM_ERR_LAYOUT, "block outside the base grid")}, log=log)
    reqs = [_request(i, shape=2 if i == 3 else 1) for i in range(6)]
    done = srv.serve(reqs, [0.0] * 6)
    assert [r.rid for r in done] == list(range(6))
    assert done[3].status == _lib.OHM_ERR_LAYOUT and "base grid" in done[3].error
    assert done[1].status == _lib.OHM_ERR_NONFINITE and "not finite" in done[1].error
    assert done[1].result is None
    assert all(done[i].status == 0 and done[i].error == "" for i in (0, 2, 4, 5))
    assert sorted(r for r, _, _ in log) == [0, 1, 2, 4, 5]
    assert all(res <= srv.budget for _, _, res in log)
    # one slot at a time; the slot of the failed solve was closed
    failed = [s for s in made if s.closed]
    assert len(failed) == 1
    assert srv.built == len(made) and srv.reused + srv.built == 5
    assert not srv.waiting and not srv.admitted
    assert srv.free == srv.budget - FP * len(srv.idle)
    srv.shutdown()
    assert srv.free == srv.budget and all(s.closed for s in made)
    rep = S.latency_report(done)
    assert rep["completed"] == 4 and rep["rejected"] == 2


@pytest.mark.timeout(60)
def test_oversized_request_is_refused_with_its_footprint(monkeypatch):
    srv = S.Server(hbm_budget=FP, n_streams=1)
    _stub(monkeypatch, srv, sizes={0: 2 * FP})
    done = srv.serve([_request(0, shape=3), _request(1)], [0.0, 0.0])
    assert done[0].status == _lib.OHM_ERR_NOMEM and str(2 * FP) in done[0].error
    assert done[1].status == 0
    srv.shutdown()
    assert srv.free == srv.budget


@pytest.mark.timeout(60)
def test_idle_slots_are_reused_and_evicted_least_recently_used_first(monkeypatch):
    """Budget of two slots, one worker, shapes A B A C A in turn: the second A
    reuses A's idle slot; C evicts B (least recently used: A was used after
    it); the last A still finds its slot."""
    srv = S.Server(hbm_budget=2 * FP, n_streams=1)
    log = []
    made = _stub(monkeypatch, srv, log=log)
    shapes = [1, 2, 1, 3, 1]
    done = srv.serve([_request(i, shape=s) for i, s in enumerate(shapes)], [0.0, 0.05, 0.10, 0.15, 0.20])
    assert all(r.status == 0 for r in done)
    assert [r.slot_reused for r in done] == [False, False, True, False, True]
    assert len(made) == 3 and srv.built == 3 and srv.reused == 2
    by_shape = {s.key[0][0]: s for s in made}
    assert by_shape[2].closed and not by_shape[1].closed and not by_shape[3].closed
    assert all(res <= srv.budget for _, _, res in log)
    srv.shutdown()
    assert srv.free == srv.budget
