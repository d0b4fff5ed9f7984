"""Benchmark: solved cells/s of Crank-Nicolson steps on one MI355X.

Workload: 128^3 periodic box, resistivity log-normal over 4 decades, div-free
random B with a k^-2 spectrum, dt = 100x the explicit limit, consecutive CN
steps each solved to a relative FP64 residual of 1e-10.  One bench step is one
CN step (the whole solve).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import statistics
import os
import sys
import time

import numpy as np

METRIC = "solved cells/s per CN step at rel. residual 1e-10 (FP64 vs mixed); HBM GB/s"
HBM_PEAK_GBS = 8000.0
# Cycle schedules (pre, post sweeps on the base grid; one sweep on the levels
# below it) picked by the autotuner on MI355X, per precision of the cycle, for
# the 128^3 log-normal workload, and for the two-level AMR workload
SCHEDULE = {0: (2, 5), 1: (2, 5)}
REPEATS = 5                 # timed blocks of the kernel rates (median)
NU_COARSE = 1
AMR_SCHEDULE = (4, 4)
SERVE_SCHEDULE = (2, 2, 0)   # (pre, post, below the base grid; 0 = as the base grid) for serving


def kernel_source_hash() -> str:
    """Hash of the sources of the block-level stencil kernels (the block
    kernels, the sweep body and the stencil they use); the counter traffic
    recorded under profiles/ is valid only for that source."""
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1009_0798_amd", "csrc")
    body = "".join(open(os.path.join(csrc, f)).read() for f in ("k_block.hip", "sweep.h", "stencil.h"))
    return hashlib.sha256(body.encode()).hexdigest()[:16]


# kernels whose HBM traffic --record-counters extracts from the counter runs of
# --roofline-only: tag -> (kernel name prefix, algorithmic bytes per cell,
# dispatches to average: the first k of that name, or all when None)
COUNTED = {
    "sweep_f64": ("k_blk_sweep<double, 0, false, true>", 80, 12),
    "sweep_f32": ("k_blk_sweep<float, 0, false, false>", 40, 12),
    "apply_f64": ("k_blk_stencil<double, 0>", 56, 12),
    "resid_f64": ("k_blk_stencil<double, 1>", 80, 12),
    "resid_restrict_f64": ("k_blk_stencil<double, 3>", 59, None),
}


def counter_traffic(tag: str, n: int):
    """HBM bytes per launch of kernel `tag` on the n^3 level-0 blocks from the
    committed counter runs (FETCH_SIZE and WRITE_SIZE, calibrated on a 256 MiB
    device copy), or None if none were taken at that size or the kernel
    source changed since."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(root, "profiles", "roofline_counters.json")) as f:
            rec = json.load(f)["kernels"][f"{tag}@{n}"]
    except (OSError, KeyError, ValueError):
        return None
    return rec["hbm_bytes"] if rec["source_sha256_16"] == kernel_source_hash() else None


def record_counters(fetch_dir: str, write_dir: str, n: int) -> dict:
    """Add to profiles/roofline_counters.json the per-launch traffic of the
    COUNTED kernels at n^3 from the two rocprofv3 --pmc runs of
    `bench.py --roofline-only --n n` (FETCH_SIZE, then WRITE_SIZE): the
    256 MiB device copy calibrates each counter."""
    import csv
    import glob
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "roofline_counters.json")

    def per_kernel(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        rows.sort()
        return rows

    copy_kib = 256 * 1024
    try:
        out = json.load(open(path))
        out["kernels"] = {k: v for k, v in out.get("kernels", {}).items() if "@" in k}
    except (OSError, ValueError):
        out = {"kernels": {}}
    cal, res = {"copy_KiB": copy_kib}, {}
    for tag, d, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        rows = per_kernel(d, counter)
        c = next(v for _, k, v in rows if "copyBuffer" in k)   # the probe's first kernel after its fill
        cal[f"{tag}_read_KiB"] = c
        cal[f"{tag}_factor"] = copy_kib / c
        res[tag] = (rows, copy_kib / c)
    out["calibration"] = cal
    cells = n ** 3
    for name, (prefix, bpc, first) in COUNTED.items():
        rec = {"kernel": prefix, "cells": cells, "source_sha256_16": kernel_source_hash(),
               "algorithmic_bytes": bpc * cells}
        tot = 0.0
        for tag in ("fetch", "write"):
            rows, factor = res[tag]
            xs = [v for _, k, v in rows if prefix in k]
            if first:
                xs = xs[:first]
            if not xs:
                break
            rec[f"{tag}_KiB"] = sum(xs) / len(xs)
            rec["dispatches"] = len(xs)
            tot += rec[f"{tag}_KiB"] * factor * 1024
        else:
            rec["hbm_bytes"] = tot
            rec["ratio"] = tot / rec["algorithmic_bytes"]
            out["kernels"][f"{name}@{n}"] = rec
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return out


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_steps(ohm, H, B0, E, dt, K, precision, ws):
    import torch
    B = [B0.clone()]
    opts = ohm.default_opts(rtol=1e-10, precision=precision, max_iters=200, nu_pre=SCHEDULE[precision][0],
                            nu_post=SCHEDULE[precision][1], nu_coarse=NU_COARSE)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        st, stats = ohm.ohm_cn_step(H, B, [E], dt, opts, ws)
        if st != 0:
            raise RuntimeError(f"CN step failed with status {st}: {stats}")
        iters.append(stats[0]["iters"])
    torch.cuda.synchronize()
    return time.perf_counter() - t0, B[0], iters, stats


def smoother_rate(ohm, H, B, S, E, lam_dt, dtype, nsweeps=10):
    """Duration of one smoother launch on the level-0 blocks (one fused
    red-black sweep per launch on a complete periodic level), measured with
    HIP events on the stream the library launches on: the median over
    REPEATS blocks of the per-launch average of `nsweeps` launches."""
    import torch
    Bt = B.to(dtype).clone()
    St = S.to(dtype).contiguous()
    Et = E.to(dtype).contiguous()
    tmp = torch.empty_like(Bt)
    ohm.ohm_smooth(H, 0, Bt, St, Et, lam_dt, 2, tmp)        # warm
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(REPEATS):
        ev0.record()
        ohm.ohm_smooth(H, 0, Bt, St, Et, lam_dt, nsweeps, tmp)
        ev1.record()
        torch.cuda.synchronize()
        runs.append(ev0.elapsed_time(ev1) / 1e3 / nsweeps)
    return statistics.median(runs)


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_steps(n_sample, min_seconds):
    """Consecutive CN steps of the oracle (FP64, V(2,2)-preconditioned
    BiCGStab to 1e-10) on the n_sample^3 log-normal workload (4 decades,
    dt = 100x explicit), as many as fit in about min_seconds (at least one).
    Returns (cells/s, steps, iterations, seconds, threads)."""
    import ohm_inputs as gen
    from oracle import mg, ref
    c = gen.config_lognormal128(n_sample)
    B = c["B"]
    steps = iters = 0
    t0 = time.perf_counter()
    while True:
        B, hist = mg.cn_step(B, c["eta"], c["spec"].dx0, c["dt"], rtol=1e-10)
        steps += 1
        iters += len(hist) - 1
        t = time.perf_counter() - t0
        if t >= min_seconds or t * (steps + 1) / steps > 3 * min_seconds:
            break
    return steps * n_sample ** 3 / t, steps, iters, t, ref.threads()


def cpu_baseline(n_sample, min_seconds=8.0, repeats=3, n_single=32):
    """The oracle timed on the host: the median of `repeats` runs with every
    host thread on the n_sample^3 sample, and one run limited to one thread
    (OpenMP and BLAS) on the n_single^3 sample."""
    from threadpoolctl import threadpool_limits
    from oracle import ref
    runs = [oracle_steps(n_sample, min_seconds) for _ in range(repeats)]
    runs.sort(key=lambda r: r[0])
    v, steps, iters, t, thr = runs[len(runs) // 2]
    nthr = ref.threads()
    ref.set_threads(1)
    try:
        with threadpool_limits(limits=1):
            single = oracle_steps(n_single, min_seconds)
    finally:
        ref.set_threads(nthr)
    return {"value": v, "unit": "cells/s", "cores": thr, "kind": "oracle",
            "sample": f"{steps} consecutive CN steps of the {n_sample}^3 log-normal workload (eta 4 decades, dt 100x "
                      f"explicit), FP64 V(2,2)-BiCGStab to 1e-10, {iters} iterations, {t:.1f} s; median of "
                      f"{repeats} runs",
            "runs_cells_per_s": [r[0] for r in runs], "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": single[0], "unit": "cells/s", "cores": single[4],
                              "sample": f"{single[1]} consecutive CN steps of the {n_single}^3 log-normal workload, "
                                        f"{single[2]} iterations, {single[3]:.1f} s"}}


def timed_oracle(make_work, min_seconds=8.0, repeats=3):
    """A bounded oracle sample: make_work() returns a function that runs one
    unit of oracle work (a CN step, or one problem) and returns (cells,
    iterations); units run until about min_seconds.  The median of `repeats`
    runs on every host thread, and one run limited to one thread (OpenMP and
    BLAS).  Returns (median, runs, single), each run (cells/s, units, cells,
    iterations, seconds, threads)."""
    from threadpoolctl import threadpool_limits
    from oracle import ref

    def one():
        work = make_work()
        units = cells = iters = 0
        t0 = time.perf_counter()
        while True:
            c, it = work()
            units += 1
            cells += c
            iters += it
            t = time.perf_counter() - t0
            if t >= min_seconds or t * (units + 1) / units > 3 * min_seconds:
                break
        return cells / t, units, cells, iters, t, ref.threads()

    runs = sorted((one() for _ in range(repeats)), key=lambda r: r[0])
    nthr = ref.threads()
    ref.set_threads(1)
    try:
        with threadpool_limits(limits=1):
            single = one()
    finally:
        ref.set_threads(nthr)
    return runs[len(runs) // 2], runs, single


def oracle_baseline(make_work, what, unit_name, min_seconds=8.0):
    """timed_oracle() as a cpu_baseline record; `what` names the sample."""
    med, runs, single = timed_oracle(make_work, min_seconds)
    return {"value": med[0], "unit": "cells/s", "cores": med[5], "kind": "oracle",
            "sample": f"{med[1]} {unit_name} of {what}, {med[2]} cells, {med[3]} iterations, {med[4]:.1f} s; median "
                      f"of {len(runs)} runs",
            "runs_cells_per_s": [r[0] for r in runs], "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "single_thread": {"value": single[0], "unit": "cells/s", "cores": single[5],
                              "sample": f"{single[1]} {unit_name}, {single[3]} iterations, {single[4]:.1f} s"}}


def bench_fourier32(args):
    """32^3, eta = 1, three axis-aligned Fourier modes plus noise, dt = 20x
    explicit: consecutive CN steps in FP64 and mixed precision, and the
    oracle on the same workload."""
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    from oracle import mg
    cfg = gen.config_fourier32()
    spec = cfg["spec"]
    ijk = spec.levels[0]
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B0 = ohm.to_blocks(torch.from_numpy(cfg["B"]), ijk).cuda()
    E = ohm.to_blocks(torch.from_numpy(cfg["eta"])[None], ijk).cuda()
    cells = spec.cells(0)[0] ** 3
    res = {}
    for prec in (0, 1):
        ws = ohm.Workspace()
        opts = ohm.default_opts(rtol=1e-10, precision=prec, max_iters=200, nu_pre=SCHEDULE[prec][0],
                                nu_post=SCHEDULE[prec][1], nu_coarse=NU_COARSE)
        B = B0.clone()
        for _ in range(args.warmup):
            ohm.ohm_cn_step(H, [B], [E], cfg["dt"], opts, ws)
        B = B0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = []
        for _ in range(args.steps):
            st, stats = ohm.ohm_cn_step(H, [B], [E], cfg["dt"], opts, ws)
            assert st == 0, st
            iters.append(stats[0]["iters"])
        torch.cuda.synchronize()
        res[prec] = ((time.perf_counter() - t0) / args.steps, iters)
    t, iters = res[0]

    def make_work():
        state = {"B": cfg["B"]}

        def work():
            state["B"], hist = mg.cn_step(state["B"], cfg["eta"], spec.dx0, cfg["dt"], rtol=1e-10)
            return cells, len(hist) - 1
        return work

    out = {"metric": METRIC, "value": cells / t, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "fourier32: 32^3, eta = 1, three Fourier modes + 1e-3 noise, dt = 20x explicit, "
                                  "consecutive CN steps to rel. residual 1e-10", "cells": cells,
                      "iterations_per_step": iters},
           "mixed": {"value": cells / res[1][0], "ms_per_step": res[1][0] * 1e3, "iterations_per_step": res[1][1]}}
    if args.cpu_sample:
        _log("timing the oracle on the same workload")
        out["cpu_baseline"] = oracle_baseline(make_work, "the 32^3 Fourier workload (the workload itself), FP64 "
                                              "V(2,2)-BiCGStab to 1e-10", "consecutive CN steps")
    return out


def bench_batched(args):
    """256 independent problems of uneven size in one handle (one launch per
    kernel covers every problem); mixed precision; schedule from the tuner."""
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    from paper_1009_0798_amd import tune
    probs = gen.config_batched(nprob=args.nprob)
    H = ohm.Hierarchy([(p["spec"].base_blocks, p["spec"].dx0, p["spec"].levels) for p in probs])
    B0 = torch.cat([ohm.to_blocks(torch.from_numpy(p["B"]), p["spec"].levels[0]) for p in probs], dim=1).cuda()
    E = torch.cat([ohm.to_blocks(torch.from_numpy(p["eta"])[None], p["spec"].levels[0]) for p in probs], dim=1).cuda()
    dts = [p["dt"] for p in probs]
    cells = sum(p["spec"].cells(0)[0] ** 3 for p in probs)
    best, table = tune.tune(H, [B0], [E], dts, finest_dx=min(p["spec"].dx0 for p in probs), precisions=(1,),
                            use_cache=False, log=_log, quick=True)
    ws = ohm.Workspace()
    opts = ohm.default_opts(rtol=1e-10, max_iters=200, **best)
    for _ in range(args.warmup):
        ohm.ohm_cn_step(H, [B0.clone()], [E], dts, opts, ws)
    Bs = [B0.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st, stats = ohm.ohm_cn_step(H, [Bs[k]], [E], dts, opts, ws)
        assert st == 0, st
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    worst = max(s["rel_res"] for s in stats)
    out = {"metric": METRIC, "value": cells * args.steps / t, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": t / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32 multigrid + f64 outer", "data": "synthetic",
            "config": {"workload": f"batched{args.nprob}: {args.nprob} independent CN solves, edges from "
                                   "{16,24,32,48,64}, eta log-normal 2 decades, dt 10-200x explicit",
                       "cells": cells, "schedule": best, "worst_rel_res": worst}}
    if args.cpu_sample:
        from oracle import mg
        _log("timing the oracle on the batch's problems in order")

        def make_work():
            it = iter(probs)

            def work():
                p = next(it)
                _, hist = mg.cn_step(p["B"], p["eta"], p["spec"].dx0, p["dt"], rtol=1e-10)
                return p["spec"].cells(0)[0] ** 3, len(hist) - 1
            return work

        out["cpu_baseline"] = oracle_baseline(make_work, "the batch (one CN step each, taken in order), FP64 "
                                              "V(2,2)-BiCGStab to 1e-10", "problems")
    return out


def bench_amr(args):
    """Two-level hierarchy: 64^3 base, central 1/8 plus a seeded 20% of the
    other base blocks refined; dense-core eta; FP64 and mixed."""
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    spec = gen.config_amr2(n_base=64, extra_frac=0.2, seed=4)
    Bb, eb = gen.amr_fields_fourier(spec, seed=5)
    dt = 20.0 * spec.dx(1) ** 2 / (6 * 10.0)
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B0 = [torch.from_numpy(b).cuda() for b in Bb]
    E = [torch.from_numpy(e[None]).cuda() for e in eb]
    cells = spec.leaf_cells()
    out = {}
    for prec in (0, 1):
        ws = ohm.Workspace()
        opts = ohm.default_opts(rtol=1e-10, max_iters=300, precision=prec, nu_pre=args.nu or AMR_SCHEDULE[0],
                                nu_post=args.nu or AMR_SCHEDULE[1], nu_coarse=NU_COARSE)
        for _ in range(args.warmup):
            ohm.ohm_cn_step(H, [b.clone() for b in B0], E, dt, opts, ws)
        Bs = [[b.clone() for b in B0] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            st, stats = ohm.ohm_cn_step(H, Bs[k], E, dt, opts, ws)
            assert st == 0, st
        torch.cuda.synchronize()
        out[prec] = ((time.perf_counter() - t0) / args.steps, stats[0])
    t, stats = out[0]
    res = {"metric": METRIC, "value": cells / t, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "amr2: 64^3 base + level 1 over the central 1/8 and 20% of other base blocks, "
                                  "dense-core eta, dt = 20x explicit on the fine level", "leaf_cells": cells,
                      "iterations": stats["iters"], "V": [args.nu or AMR_SCHEDULE[0], args.nu or AMR_SCHEDULE[1]]},
           "mixed": {"value": cells / out[1][0], "ms_per_step": out[1][0] * 1e3, "iterations": out[1][1]["iters"]}}
    if args.cpu_sample:
        from oracle import amr
        _log("timing the oracle's composite step on the 32^3-base version of the workload")
        sspec = gen.config_amr2(n_base=32, extra_frac=0.2, seed=4)
        sb, se = gen.amr_fields_fourier(sspec, seed=5)
        sdt = 20.0 * sspec.dx(1) ** 2 / (6 * 10.0)
        C = amr.Composite(sspec)
        e = [C.to_dense(l, se[l]) for l in range(2)]

        def make_work():
            state = {"b": [C.to_dense(l, sb[l]) for l in range(2)]}

            def work():
                state["b"], hist = C.cn_step(state["b"], e, sdt, rtol=1e-10)
                return sspec.leaf_cells(), len(hist) - 1
            return work

        res["cpu_baseline"] = oracle_baseline(
            make_work, f"the same recipe on a 32^3 base ({sspec.leaf_cells()} leaf cells; the 64^3-base step takes "
                       "about a minute on the oracle), composite operator with point-Jacobi BiCGStab to 1e-10",
            "consecutive CN steps")
    return res


def bench_serve(args):
    """Poisson arrivals of 1-3 level AMR requests (a pool of request shapes,
    reused), continuous batching over resident slots: the offered rate, then
    a rate below the measured capacity (the sustainable one), each with
    p50 / p99 latency."""
    import numpy as np
    import ohm_inputs as gen
    from paper_1009_0798_amd.serve import Request, Server, latency_report, poisson_arrivals
    rng = np.random.default_rng(7)
    pool = []
    for i in range(args.pool):
        n0 = int(rng.choice(np.arange(32, 193, 8)))
        L = int(rng.choice([1, 2, 3]))
        d = gen.amr_request(rng, n0, L, float(rng.uniform(0, 4)), float(np.exp(rng.uniform(np.log(10), np.log(100)))))
        pool.append(d)
        _log(f"request template {i}: base {n0}^3, levels {d['spec'].nlevels}, leaf cells {d['spec'].leaf_cells()}")

    def requests(n, first):
        out = []
        for i in range(n):
            d = pool[(first + i) % len(pool)]
            s = d["spec"]
            out.append(Request(rid=first + i, arrival=0.0, base_blocks=s.base_blocks, dx0=s.dx0, levels=s.levels,
                               B=d["B"], eta=d["eta"], dt=d["dt"]))
        return out

    sched = dict(zip(("nu_pre", "nu_post", "nu_coarse"), SERVE_SCHEDULE))
    srv = Server(hbm_budget=int(args.hbm_gb * (1 << 30)), n_streams=args.streams, **sched)
    # one pass over the pool first (untimed): every shape gets its slot
    srv.serve(requests(len(pool), 10 ** 6), [0.0] * len(pool))
    legs = {}
    rate = args.rate
    for name in ("offered", "sustainable"):
        srv.finished = []
        reqs = requests(args.requests, 0)
        done = srv.serve(reqs, poisson_arrivals(rate, len(reqs), seed=7))
        rep = latency_report(done)
        rep["rate_per_s"] = rate
        legs[name] = rep
        _log(f"{name}: {rate:.1f}/s offered, {rep['requests_per_s']:.1f}/s served, p50 {rep['p50_ms']:.0f} ms, "
             f"p99 {rep['p99_ms']:.0f} ms, {rep['cells_per_s']:.3e} cells/s")
        rate = 0.8 * rep["requests_per_s"]
    srv.shutdown()
    rep = legs["offered"]
    out = {"metric": METRIC, "value": rep["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": args.requests,
           "warmup": len(pool), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 multigrid + f64 outer", "data": "synthetic",
           "config": {"workload": f"serve: Poisson {args.rate}/s, {args.requests} requests of 1-3 level AMR, base "
                                  "32-192^3", "streams": args.streams, "schedule": sched},
           "latency": rep, "sustainable": legs["sustainable"],
           "slots": {"built": srv.built, "reused": srv.reused}}
    if args.cpu_sample:
        from oracle import amr
        limit = 200_000
        small = sorted((d for d in pool if d["spec"].leaf_cells() <= limit), key=lambda d: d["spec"].leaf_cells())
        if small:
            _log("timing the oracle's composite step on the smallest request shapes")

            def make_work():
                it = iter(small * 100)

                def work():
                    d = next(it)
                    C = amr.Composite(d["spec"])
                    L = d["spec"].nlevels
                    b = [C.to_dense(l, d["B"][l]) for l in range(L)]
                    e = [C.to_dense(l, d["eta"][l]) for l in range(L)]
                    _, hist = C.cn_step(b, e, d["dt"], rtol=1e-10)
                    return d["spec"].leaf_cells(), len(hist) - 1
                return work

            cb = oracle_baseline(make_work, f"the pool's request shapes with at most {limit} leaf cells, smallest "
                                            f"first ({[d['spec'].leaf_cells() for d in small]} leaf cells; the "
                                            "others take minutes each), one composite step each, point-Jacobi "
                                            "BiCGStab to 1e-10", "requests")
            out["cpu_baseline"] = cb
    return out


def bench_e8(args):
    """The comparison of section 3.3 at its own size: 64^3 on [-4, 4)^3,
    eta = exp(-r^2), B_z = exp(-(x^2 + y^2)), to t = 1: the explicit
    predictor-corrector scheme with dt = 1e-3 (1000 steps) against the implicit
    scheme with dt = 0.1 (10 steps, lambda = 1/2 and 1), FP64.  Reports the
    time to solution of each and their differences."""
    import numpy as np
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    cfg = gen.config_e8(64)
    spec = cfg["spec"]
    ijk = spec.levels[0]
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B0 = ohm.to_blocks(torch.from_numpy(cfg["B"]), ijk).cuda()
    E = [ohm.to_blocks(torch.from_numpy(cfg["eta"])[None], ijk).cuda()]
    nexp = int(round(cfg["t_end"] / cfg["dt_explicit"]))
    nimp = int(round(cfg["t_end"] / cfg["dt_implicit"]))
    ws = ohm.Workspace()
    ohm.ohm_explicit_step(H, [B0.clone()], E, cfg["dt_explicit"], 10, ws)      # warm
    Bx = B0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ohm.ohm_explicit_step(H, [Bx], E, cfg["dt_explicit"], nexp, ws)
    torch.cuda.synchronize()
    t_exp = time.perf_counter() - t0
    out = {"explicit": {"steps": nexp, "dt": cfg["dt_explicit"], "seconds": t_exp}}
    for lam in (0.5, 1.0):
        opts = ohm.default_opts(rtol=1e-10, max_iters=200, lam=lam)
        ohm.ohm_cn_step(H, [B0.clone()], E, cfg["dt_implicit"], opts, ws)        # warm
        Bi = B0.clone()
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nimp):
            st, stats = ohm.ohm_cn_step(H, [Bi], E, cfg["dt_implicit"], opts, ws)
            assert st == 0, st
            its.append(stats[0]["iters"])
        torch.cuda.synchronize()
        t_imp = time.perf_counter() - t0
        diff = float(torch.linalg.vector_norm(Bi - Bx) / torch.linalg.vector_norm(Bx))
        out[f"implicit_lambda_{lam}"] = {"steps": nimp, "dt": cfg["dt_implicit"], "seconds": t_imp,
                                         "iterations": its, "rel_diff_vs_explicit": diff}
        _log(f"lambda {lam}: {t_imp * 1e3:.1f} ms for {nimp} steps, rel. diff. vs explicit {diff:.2e}")
    _log(f"explicit: {t_exp * 1e3:.1f} ms for {nexp} steps")
    cells = spec.cells(0)[0] ** 3
    return {"metric": METRIC, "value": cells * nimp / out["implicit_lambda_0.5"]["seconds"], "unit": "cells/s",
            "n_gpus": 1, "steps": nimp, "warmup": 1, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "e8: section 3.3 comparison, 64^3 on [-4,4)^3, eta = exp(-r^2), "
                                   "B_z = exp(-(x^2+y^2)), t = 1", "cells": cells},
            "comparison": out,
            "speedup_to_solution_vs_explicit": t_exp / out["implicit_lambda_0.5"]["seconds"]}


def stencil_rate(ohm, H, B, S, E, coef, kind, nlaunch=10):
    """Duration of one launch of the level-0 operator apply (out = B + coef
    div F(B)) or residual (R = S - L B, no norms), measured with HIP events
    on the stream the library launches on: the median over REPEATS blocks of
    the per-launch average of `nlaunch` launches."""
    import torch
    out = torch.empty_like(B)

    def once():
        if kind == "apply":
            ohm.ohm_apply(H, 0, B, E, coef, out)
        else:
            ohm.ohm_residual(H, 0, B, S, E, coef, R=out)

    once()
    once()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(REPEATS):
        ev0.record()
        for _ in range(nlaunch):
            once()
        ev1.record()
        torch.cuda.synchronize()
        runs.append(ev0.elapsed_time(ev1) / 1e3 / nlaunch)
    return statistics.median(runs)


def random_level(n, seed=11):
    """Hierarchy and resident level-0 fields of an n^3 periodic box filled on
    the device with seeded random values (B, S standard normal, eta
    log-uniform over 4 decades): the stencil kernels' timing does not depend on
    the values."""
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    spec = gen.uniform_spec(n)
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    nb = len(spec.levels[0])
    B = torch.randn((3, nb, 8, 8, 8), dtype=torch.float64, device="cuda", generator=g)
    S = torch.randn((3, nb, 8, 8, 8), dtype=torch.float64, device="cuda", generator=g)
    E = 10.0 ** (-4.0 * torch.rand((1, nb, 8, 8, 8), dtype=torch.float64, device="cuda", generator=g))
    return spec, H, B, S, E, gen.explicit_dt(spec.dx0, 1.0, 100.0)


def roofline_probe(args):
    """For the counter runs: a plain device copy of 256 MiB (calibrates the
    HBM byte counters), then on the level-0 blocks of the n^3 log-normal
    workload 12 launches each of the FP64 and FP32 fused sweeps, the FP64
    operator apply and the FP64 residual, then one FP64 CN step (its residual
    with restriction to the first coarse level)."""
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    cfg = gen.config_lognormal128(args.n)
    spec = cfg["spec"]
    ijk = spec.levels[0]
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B0 = ohm.to_blocks(torch.from_numpy(cfg["B"]), ijk).cuda()
    E = ohm.to_blocks(torch.from_numpy(cfg["eta"])[None], ijk).cuda()
    S = torch.randn_like(B0)
    lam_dt = 0.5 * cfg["dt"]
    for dt in (torch.float64, torch.float32):
        t = smoother_rate(ohm, H, B0, S, E, lam_dt, dt, nsweeps=10)
        _log(f"smoother {dt}: {t * 1e6:.2f} us per launch")
    for kind in ("apply", "resid"):
        t = stencil_rate(ohm, H, B0, S, E, lam_dt, kind)
        _log(f"{kind} float64: {t * 1e6:.2f} us per launch")
    opts = ohm.default_opts(rtol=1e-10, max_iters=200, nu_pre=SCHEDULE[0][0], nu_post=SCHEDULE[0][1],
                            nu_coarse=NU_COARSE)
    st, stats = ohm.ohm_cn_step(H, [B0.clone()], [E], cfg["dt"], opts)
    _log(f"cn step: status {st}, {stats[0]['iters']} iterations")
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--cpu-sample", type=int, default=64, help="grid edge of the oracle sample (0: skip)")
    ap.add_argument("--hbm-n", type=int, default=256,
                    help="grid edge of the second roofline leg, a working set above the last-level cache (0: skip)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--workload", default="lognormal128", choices=["lognormal128", "fourier32", "batched", "serve", "amr", "e8"])
    ap.add_argument("--nu", type=int, default=None, help="pre and post sweeps of the AMR workload's cycle")
    ap.add_argument("--nprob", type=int, default=256)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--pool", type=int, default=8)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--record-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="add to profiles/roofline_counters.json the kernels' traffic at --n from two rocprofv3 --pmc "
                         "runs of --roofline-only --n")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only a known-size copy and the level-0 stencil kernels at --n (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm

    if args.record_counters:
        print(json.dumps(record_counters(*args.record_counters, args.n), indent=1))
        return
    if args.roofline_only:
        roofline_probe(args)
        return
    if args.workload == "e8":
        print(json.dumps(bench_e8(args)), flush=True)
        return
    if args.workload == "fourier32":
        print(json.dumps(bench_fourier32(args)), flush=True)
        return
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "amr":
        print(json.dumps(bench_amr(args)), flush=True)
        return
    n = args.n
    cfg = gen.config_lognormal128(n)
    spec = cfg["spec"]
    ijk = spec.levels[0]
    _log(f"workload {n}^3, dt={cfg['dt']:.4e}")
    H = ohm.Hierarchy([(spec.base_blocks, spec.dx0, spec.levels)])
    B0 = ohm.to_blocks(torch.from_numpy(cfg["B"]), ijk).cuda()
    E = ohm.to_blocks(torch.from_numpy(cfg["eta"])[None], ijk).cuda()
    ws = ohm.Workspace()
    cells = n ** 3
    res = {}
    for prec, name in ([(0, "f64")] + ([] if args.no_mixed else [(1, "mixed")])):
        if args.warmup:
            run_steps(ohm, H, B0, E, cfg["dt"], args.warmup, prec, ws)
        t, Bend, iters, stats = run_steps(ohm, H, B0, E, cfg["dt"], args.steps, prec, ws)
        res[name] = dict(t=t, B=Bend, iters=iters, rel_res=stats[0]["rel_res"])
        _log(f"{name}: {t / args.steps * 1e3:.2f} ms/step, iterations {iters}, rel_res {stats[0]['rel_res']:.2e}")

    f64 = res["f64"]
    value = cells * args.steps / f64["t"]
    # roofline of the dominant kernel, the fused red-black sweep on the
    # level-0 blocks: on the workload itself, whose 168 MB sweep working set
    # fits the 256 MB last-level cache, and on a 256^3 level (1.34 GB) that
    # streams from HBM
    S = torch.randn_like(B0)
    lam_dt = 0.5 * cfg["dt"]
    t_sw = smoother_rate(ohm, H, B0, S, E, lam_dt, torch.float64)
    bytes_sw = cells * 10 * 8          # read B, S, eta (7 values), write B (3) per cell
    achieved = bytes_sw / t_sw / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": f64["t"] / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"lognormal{n}: {n}^3 periodic, eta log-normal 4 decades, div-free k^-2 B, "
                               f"dt = 100x explicit limit, consecutive CN steps to rel. residual 1e-10",
                   "cells": cells, "outer": "BiCGStab",
                   "cycle": f"V{SCHEDULE[0]} (FP64) / V{SCHEDULE[1]} (mixed), {NU_COARSE} sweep below the base grid",
                   "iterations_per_step": f64["iters"]},
        "roofline": {"kernel": "k_blk_sweep<double> (one fused red-black sweep, level 0)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic("sweep_f64", n),
                     "us_per_launch": t_sw * 1e6, "bytes_per_launch": bytes_sw,
                     "timing": f"median of {REPEATS} blocks of 10 launches (HIP events on the library's stream)",
                     "residency": f"{n}^3: {bytes_sw / 1e6:.0f} MB working set"
                                  + (", inside the 256 MB last-level cache" if bytes_sw < 256e6 else "")},
    }
    if args.hbm_n:
        nh = args.hbm_n
        _, Hh, Bh, Sh, Eh, dth = random_level(nh)
        ch = nh ** 3
        t_h = smoother_rate(ohm, Hh, Bh, Sh, Eh, 0.5 * dth, torch.float64)
        leg = {"kernel": "k_blk_sweep<double> (one fused red-black sweep, level 0)", "bound": "hbm",
               "achieved": ch * 80 / t_h / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": ch * 80 / t_h / 1e9 / HBM_PEAK_GBS, "traffic": counter_traffic("sweep_f64", nh),
               "us_per_launch": t_h * 1e6, "bytes_per_launch": ch * 80,
               "timing": f"median of {REPEATS} blocks of 10 launches (HIP events on the library's stream)",
               "residency": f"{nh}^3: {ch * 80 / 1e9:.2f} GB working set, streamed from HBM", "others": {}}
        for kind, tag, bpc in (("apply", "apply_f64", 56), ("resid", "resid_f64", 80)):
            t_k = stencil_rate(ohm, Hh, Bh, Sh, Eh, 0.5 * dth, kind)
            leg["others"][tag] = {"us_per_launch": t_k * 1e6, "bytes_per_launch": ch * bpc,
                                  "achieved": ch * bpc / t_k / 1e9, "frac": ch * bpc / t_k / 1e9 / HBM_PEAK_GBS,
                                  "traffic": counter_traffic(tag, nh)}
        out["roofline_hbm"] = leg
        _log(f"{nh}^3 sweep: {t_h * 1e6:.1f} us per launch, {leg['achieved']:.0f} GB/s algorithmic")
        del Hh, Bh, Sh, Eh
    if "mixed" in res:
        mx = res["mixed"]
        diff = (mx["B"] - f64["B"]).norm().item() / f64["B"].norm().item()
        t32 = smoother_rate(ohm, H, B0, S, E, lam_dt, torch.float32)
        out["mixed"] = {"value": cells * args.steps / mx["t"], "ms_per_step": mx["t"] / args.steps * 1e3,
                        "dtype": "f32 multigrid + f64 outer", "iterations_per_step": mx["iters"],
                        "rel_diff_vs_f64_after_steps": diff,
                        "smoother_f32_GBs": cells * 10 * 4 / t32 / 1e9}
    if args.cpu_sample:
        _log(f"timing the oracle on a {args.cpu_sample}^3 sample")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
