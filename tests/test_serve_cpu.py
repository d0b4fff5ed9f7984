"""Host logic of the request server, without a GPU: the sizing of a request
and the solve of a batch are replaced by stand-ins, so what runs is the
admission, batching and failure handling alone."""
import numpy as np
import pytest

from paper_1009_0798_amd import _lib
from paper_1009_0798_amd import serve as S

FP = 10


def _requests(n):
    return [S.Request(rid=i, arrival=0.0, base_blocks=(1, 1, 1), dx0=0.125,
                      levels=[np.zeros((1, 3), np.int32)], B=[np.zeros((3, 1, 8, 8, 8))],
                      eta=[np.ones((1, 8, 8, 8))], dt=1.0) for i in range(n)]


@pytest.mark.timeout(60)
def test_failures_finish_their_requests_and_return_the_budget(monkeypatch):
    """Request 3 is refused at sizing (as the library refuses blocks outside
    the base grid), request 1's batch raises inside the solve.  With a budget
    of one request at a time, a batch whose budget were lost would starve every
    later request; instead all six finish, the two failures with their
    library status and message, and the whole budget is free at the end."""
    def footprint(req, opts):
        if req.rid == 3:
            raise _lib.OhmError(_lib.OHM_ERR_LAYOUT, "block outside the base grid")
        return FP

    srv = S.Server(hbm_budget=FP, n_streams=2, max_batch=1)
    srv.streams = [None, None]
    seen = []

    def run_batch(batch, stream, ws):
        seen.append([r.rid for r in batch])
        assert srv.budget - srv.free == FP * len(batch)
        if any(r.rid == 1 for r in batch):
            raise _lib.OhmError(_lib.OHM_ERR_NONFINITE, "eta is not finite")
        for r in batch:
            r.status, r.result, r.done = 0, [], srv.now()

    monkeypatch.setattr(S, "footprint", footprint)
    monkeypatch.setattr(srv, "_run_batch", run_batch)
    done = srv.serve(_requests(6), [0.0] * 6)
    assert [r.rid for r in done] == list(range(6))
    assert done[3].status == _lib.OHM_ERR_LAYOUT and "base grid" in done[3].error
    assert done[1].status == _lib.OHM_ERR_NONFINITE and "not finite" in done[1].error
    assert done[1].result is None
    assert all(done[i].status == 0 and done[i].error == "" for i in (0, 2, 4, 5))
    assert sorted(sum(seen, [])) == [0, 1, 2, 4, 5]
    assert srv.free == srv.budget and not srv.waiting and not srv.admitted
    rep = S.latency_report(done)
    assert rep["completed"] == 4 and rep["rejected"] == 2


@pytest.mark.timeout(60)
def test_oversized_request_is_refused_with_its_footprint(monkeypatch):
    monkeypatch.setattr(S, "footprint", lambda req, opts: 2 * FP if req.rid == 0 else FP)
    srv = S.Server(hbm_budget=FP, n_streams=1)
    srv.streams = [None]

    def run_batch(batch, stream, ws):
        for r in batch:
            r.status, r.done = 0, srv.now()

    monkeypatch.setattr(srv, "_run_batch", run_batch)
    done = srv.serve(_requests(2), [0.0, 0.0])
    assert done[0].status == _lib.OHM_ERR_NOMEM and str(2 * FP) in done[0].error
    assert done[1].status == 0 and srv.free == srv.budget
