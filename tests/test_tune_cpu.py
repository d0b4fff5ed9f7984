"""The schedule autotuner's host logic without a GPU: candidate generation,
the choice of the fastest schedule that converges, and the cache keyed by GPU
model, problem size, eta dt / h^2 and precisions.  The step itself and the
clock are stand-ins (each candidate's step costs a known time)."""
import types

import numpy as np
import pytest
import torch

from paper_1009_0798_amd import _lib, tune


def test_candidates_cover_the_schedule_table():
    full = list(tune.candidates((0, 1)))
    quick = list(tune.candidates((1,), quick=True))
    assert len(full) == len(tune.SWEEPS) * len(tune.COARSE) * len(tune.CYCLES) * len(tune.OUTERS) * 2
    assert len(quick) == len(tune.SWEEPS) * len(tune.COARSE)
    assert all(c["cycle"] == 0 and c["outer"] == 1 and c["precision"] == 1 for c in quick)
    # every candidate is distinct and names only ohm_cn_opts fields
    keys = {tuple(sorted(c.items())) for c in full}
    assert len(keys) == len(full)
    names = {f[0] for f in _lib.CnOpts._fields_}
    assert all(set(c) <= names for c in full)


class _Clock:
    def __init__(self):
        self.t = 0.0

    def perf_counter(self):
        return self.t


def _stub(monkeypatch, cost, fails=()):
    """ohm_cn_step stand-in: a candidate's step advances the clock by
    cost(opts) and reports 3 iterations, or fails."""
    clock = _Clock()
    calls = []

    def step(h, B, eta, dt, opts, ws):
        c = dict(nu_pre=opts.nu_pre, nu_post=opts.nu_post, nu_coarse=opts.nu_coarse, cycle=opts.cycle,
                 outer=opts.outer, precision=opts.precision)
        calls.append(c)
        if tuple(sorted(c.items())) in fails:
            return _lib.OHM_ERR_NOCONV, [dict(iters=200, rel_res=1.0)]
        clock.t += cost(c)
        return 0, [dict(iters=3, rel_res=1e-11)]

    monkeypatch.setattr(tune, "ohm_cn_step", step)
    monkeypatch.setattr(tune, "time", types.SimpleNamespace(perf_counter=clock.perf_counter))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    return calls


def test_tune_picks_the_fastest_converging_schedule_and_caches_it(monkeypatch, tmp_path):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    # fastest: V(3, 4) with one coarse sweep; the only faster one fails
    best_c = dict(nu_pre=3, nu_post=4, nu_coarse=1, cycle=0, outer=1, precision=1)
    fast_fail = dict(nu_pre=1, nu_post=2, nu_coarse=0, cycle=0, outer=1, precision=1)

    def cost(c):
        if c == best_c:
            return 1.0
        return 2.0 + c["nu_pre"] + c["nu_post"] + c["nu_coarse"]

    calls = _stub(monkeypatch, cost, fails={tuple(sorted(fast_fail.items()))})
    h = types.SimpleNamespace(nprob=2)
    B = [torch.ones(3, 4, 8, 8, 8, dtype=torch.float64)]
    E = [torch.full((1, 4, 8, 8, 8), 0.5, dtype=torch.float64)]
    best, table = tune.tune(h, B, E, [1e-3, 2e-3], finest_dx=0.0625, precisions=(1,), quick=True)
    assert best == best_c
    failed = [c for c, t, _ in table if t is None]
    assert failed == [fast_fail]
    n = len(calls)
    # a second call with the same key reads the cache (no step runs)
    best2, _ = tune.tune(h, B, E, [1e-3, 2e-3], finest_dx=0.0625, precisions=(1,), quick=True)
    assert best2 == best_c and len(calls) == n
    # another eta dt / h^2 bucket is tuned again
    tune.tune(h, B, [e * 64 for e in E], [1e-3, 2e-3], finest_dx=0.0625, precisions=(1,), quick=True)
    assert len(calls) > n


def test_tune_raises_when_nothing_converges(monkeypatch, tmp_path):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    every = {tuple(sorted(c.items())) for c in tune.candidates((1,), quick=True)}
    _stub(monkeypatch, lambda c: 1.0, fails=every)
    h = types.SimpleNamespace(nprob=1)
    B = [torch.ones(3, 1, 8, 8, 8, dtype=torch.float64)]
    E = [torch.ones(1, 1, 8, 8, 8, dtype=torch.float64)]
    with pytest.raises(RuntimeError):
        tune.tune(h, B, E, 1e-3, finest_dx=0.125, precisions=(1,), quick=True, use_cache=False)
