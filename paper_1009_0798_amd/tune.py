"""Autotuner for the solver schedule of ``ohm_cn_step``.

The time of a step is (outer iterations) x (cost of one multigrid application
and one operator apply); both factors depend on the sweep counts, the cycle
(V or full multigrid), the outer iteration (BiCGStab or the iterative
multigrid of eqs. 16-18) and the precision of the cycle.  The tuner times one
step of each candidate schedule on the caller's own problem (a copy of B, so
the caller's data are untouched), keeps the fastest one that converges, and
caches the choice per GPU model, problem-size bucket and eta dt / h^2 bucket.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import Workspace, default_opts, ohm_cn_step

CACHE = os.environ.get("OHM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ohm_tune.json"))

SWEEPS = [(n1, n2) for n1 in (1, 2, 3, 4) for n2 in (2, 3, 4, 5, 6)]   # (pre, post) on the base grid
COARSE = [0, 1, 2]          # sweeps on the levels below the base grid (0 = same as the base grid)
CYCLES = [0, 1]
OUTERS = [1, 0]


def _key(h, B, eta, dt, finest_dx, precisions) -> str:
    import torch
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    cells = sum(int(b.numel()) // 3 for b in B)
    emax = max(float(e.max().item()) for e in eta)
    dts = dt if hasattr(dt, "__len__") else [dt]
    r = emax * max(dts) / finest_dx ** 2
    return f"{name}|nprob={h.nprob}|cells=2^{round(math.log2(max(cells, 1)))}|r=2^{round(math.log2(max(r, 1e-9)))}" \
           f"|prec={','.join(map(str, precisions))}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(db):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def candidates(precisions=(0, 1), quick=False):
    """Schedules to try.  quick: BiCGStab with V-cycles only (the iterative
    multigrid of eqs. 16-18 and full multigrid are far slower on every
    workload measured so far)."""
    cycles = [0] if quick else CYCLES
    outers = [1] if quick else OUTERS
    for (n1, n2), nc, cyc, outer, prec in itertools.product(SWEEPS, COARSE, cycles, outers, precisions):
        yield dict(nu_pre=n1, nu_post=n2, nu_coarse=nc, cycle=cyc, outer=outer, precision=prec)


def tune(h, B, eta, dt, finest_dx, precisions=(0, 1), rtol=1e-10, use_cache=True, repeats=1, log=None,
         quick=False):
    """Return (best option dict, table of (options, seconds, iterations)).

    ``B`` and ``eta`` are the per-level tensors of ``ohm_cn_step``; B is copied
    for every trial; ``finest_dx`` is the smallest cell width of the handle."""
    import torch
    key = _key(h, B, eta, dt, finest_dx, precisions)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return db[key]["best"], db[key]["table"]
    ws = Workspace()
    table = []
    for cand in candidates(precisions, quick):
        opts = default_opts(rtol=rtol, max_iters=200, **cand)
        Bc = [b.clone() for b in B]
        st, stats = ohm_cn_step(h, Bc, eta, dt, opts, ws)      # warm (graph capture, coarse inverse)
        if st != 0:
            table.append((cand, None, None))
            continue
        best_t = None
        for _ in range(repeats):
            Bc = [b.clone() for b in B]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, stats = ohm_cn_step(h, Bc, eta, dt, opts, ws)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best_t = t if best_t is None else min(best_t, t)
        its = max(s["iters"] for s in stats)
        table.append((cand, best_t if st == 0 else None, its))
        if log:
            log(f"tune {cand}: {best_t * 1e3:.2f} ms, {its} iterations, status {st}")
    ok = [(t, c) for c, t, _ in table if t is not None]
    if not ok:
        raise RuntimeError("no candidate schedule converged")
    best = min(ok, key=lambda x: x[0])[1]
    if use_cache:
        db[key] = {"best": best, "table": table}
        _save(db)
    return best, table
