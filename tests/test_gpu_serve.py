"""Serving: requests of mixed sizes and 1-2 AMR levels arriving over time are
admitted by footprint into resident slots, solved on several streams at once
(their outer iterations interleave), and each served result equals the same
request solved alone (bitwise: per-problem reductions in a fixed order) and
meets the FP64 residual tolerance by the oracle's composite residual."""
import dataclasses

import numpy as np
import pytest

import ohm_inputs as gen

from gpu_util import announce

pytestmark = pytest.mark.gpu


def _requests(n, seed):
    from paper_1009_0798_amd.serve import Request
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        n0 = int(rng.choice([16, 24, 32]))
        L = int(rng.choice([1, 2]))
        d = gen.amr_request(rng, n0, L, float(rng.uniform(0, 3)), float(np.exp(rng.uniform(np.log(10), np.log(60)))))
        s = d["spec"]
        out.append(Request(rid=i, arrival=0.0, base_blocks=s.base_blocks, dx0=s.dx0, levels=s.levels, B=d["B"],
                           eta=d["eta"], dt=d["dt"]))
    return out


def _alone(r, precision):
    import torch
    import paper_1009_0798_amd as ohm
    h = ohm.Hierarchy([(r.base_blocks, r.dx0, r.levels)])
    B = [torch.from_numpy(b).cuda() for b in r.B]
    E = [torch.from_numpy(e[None]).cuda() for e in r.eta]
    st, stats = ohm.ohm_cn_step(h, B, E, r.dt, ohm.default_opts(rtol=1e-10, precision=precision, max_iters=300))
    return st, stats, [b.cpu().numpy() for b in B]


@pytest.mark.parametrize("precision", [1])
def test_served_equals_alone(precision):
    from paper_1009_0798_amd.serve import Server, latency_report, poisson_arrivals
    announce("serve: served == alone")
    reqs = _requests(10, seed=71)
    srv = Server(hbm_budget=2 << 30, n_streams=3, precision=precision)
    done = srv.serve(reqs, poisson_arrivals(200.0, len(reqs), seed=7))
    # a second wave repeats three shapes (all distinct): their idle slots are reused
    again = [dataclasses.replace(reqs[i], rid=10 + k, result=None, stats=None, status=-1)
             for k, i in enumerate((0, 1, 2))]
    built = srv.built
    done = srv.serve(again, poisson_arrivals(200.0, len(again), seed=8))
    rep = latency_report(done)
    print(rep, "slots built", srv.built, "reused", srv.reused)
    assert rep["completed"] == len(reqs) + len(again)
    assert srv.built == built and srv.reused >= 3
    for r in done:
        assert r.status == 0 and r.stats["rel_res"] <= 1e-10
        st, stats, alone = _alone(r, precision)
        assert st == 0
        for l in range(len(r.levels)):
            assert np.array_equal(alone[l], r.result[l]), (r.rid, l)
        rel = _oracle_rel_residual(r)
        print(r.rid, "oracle rel. residual", rel, "library", r.stats["rel_res"])
        assert rel <= 1.01e-10


def _oracle_rel_residual(r):
    """|S - L B|_2 / |S|_2 of a served result by the oracle's composite
    operator (leaf cells of every level; S from the request's input)."""
    from oracle import amr
    spec = gen.HierSpec(tuple(r.base_blocks), r.dx0, list(r.levels))
    C = amr.Composite(spec)
    L = spec.nlevels
    b = [C.to_dense(l, r.B[l]) for l in range(L)]
    e = [C.to_dense(l, r.eta[l]) for l in range(L)]
    got = [C.to_dense(l, np.asarray(r.result[l])) for l in range(L)]
    S = C.source(b, e, r.dt)
    R = C.residual(got, S, e, 0.5 * r.dt)
    return float(np.linalg.norm(C.pack(R)) / np.linalg.norm(C.pack(S)))


def _pool_request(n0, L, seed):
    """A request of the serving workload's recipe (1-3 levels, each finer level
    one compact patch of about 1/8 of its parent, eta up to 4 decades, dt
    10-100x the finest explicit limit) at a given base size."""
    from paper_1009_0798_amd.serve import Request
    rng = np.random.default_rng(seed)
    d = gen.amr_request(rng, n0, L, float(rng.uniform(2, 4)), float(np.exp(rng.uniform(np.log(10), np.log(100)))))
    s = d["spec"]
    assert s.nlevels == L
    return Request(rid=0, arrival=0.0, base_blocks=s.base_blocks, dx0=s.dx0, levels=s.levels, B=d["B"],
                   eta=d["eta"], dt=d["dt"])


@pytest.mark.parametrize("n0,L", [(192, 1), (184, 2), (96, 3)])
def test_served_full_size_against_oracle(n0, L):
    """Full-size requests of the serving workload (base up to 192^3, 1-3
    levels), served in mixed precision: the oracle's composite residual of each
    served answer meets the tolerance (a property that holds at any size; the
    oracle's composite operator holds every level as a dense box, so the
    three-level case uses a 96^3 base, whose finest level is 384^3)."""
    from paper_1009_0798_amd.serve import Server
    announce(f"serve: full-size request base {n0}^3, {L} levels")
    r = _pool_request(n0, L, seed=700 + n0 + L)
    srv = Server(hbm_budget=64 << 30, n_streams=1, precision=1)
    done = srv.serve([r], [0.0])
    assert done[0].status == 0, done[0].error
    rel = _oracle_rel_residual(done[0])
    print("oracle rel. residual", rel, "library", done[0].stats)
    assert rel <= 1.01e-10


def test_admission_by_footprint():
    """A budget that fits one request at a time serialises them; a request
    larger than the whole budget is rejected."""
    from paper_1009_0798_amd.serve import Server, footprint
    announce("serve: admission")
    reqs = _requests(3, seed=72)
    srv = Server(hbm_budget=1, n_streams=2)
    fps = [footprint(r, srv.opts) for r in reqs]
    srv = Server(hbm_budget=max(fps), n_streams=2)
    done = srv.serve(reqs, [0.0, 0.0, 0.0])
    assert all(r.status == 0 for r in done)
    # at every admission the footprints of the resident requests fit the budget
    fp = {r.rid: f for r, f in zip(reqs, fps)}
    for r in done:
        t = r.admitted
        resident = [q for q in done if q.admitted <= t < q.done]
        assert sum(fp[q.rid] for q in resident) <= max(fps)
    # and the largest request was never resident with another one
    big = max(done, key=lambda q: fp[q.rid])
    others = [q for q in done if q is not big]
    assert all(q.done <= big.admitted + 1e-9 or q.admitted >= big.done - 1e-9 for q in others)
    tiny = Server(hbm_budget=min(fps) - 1, n_streams=1)
    done = tiny.serve(reqs[:1], [0.0])
    assert done[0].status != 0


def test_cancel_releases_budget():
    """Cancelling an admitted request frees its footprint and admits the next
    waiting one; cancelling a waiting request removes it; both are reported
    with a non-zero status and nothing is solved for them."""
    from paper_1009_0798_amd.serve import Server, footprint
    announce("serve: cancel")
    reqs = _requests(3, seed=73)
    probe = Server(hbm_budget=1, n_streams=1)
    fps = [footprint(r, probe.opts) for r in reqs]
    srv = Server(hbm_budget=max(fps), n_streams=1)
    for r in reqs:
        srv.submit(r)
    assert [r.rid for r in srv.admitted] == [0] and [r.rid for r in srv.waiting] == [1, 2]
    assert srv.free == max(fps) - fps[0]
    assert srv.cancel(0)
    assert [r.rid for r in srv.admitted] == [1] and srv.free == max(fps) - fps[1]
    assert srv.cancel(2) and not srv.waiting
    assert not srv.cancel(2)
    assert sorted(r.rid for r in srv.finished) == [0, 2] and all(r.status != 0 for r in srv.finished)
