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
import os
import sys
import time

import numpy as np

METRIC = "solved cells/s per CN step at rel. residual 1e-10 (FP64 vs mixed); HBM GB/s"
HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_steps(ohm, H, B0, E, dt, K, precision, ws):
    import torch
    B = [B0.clone()]
    opts = ohm.default_opts(rtol=1e-10, precision=precision, max_iters=200)
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
    """Average duration of one red-black half-sweep launch on the level-0
    blocks, measured with HIP events on the stream the library launches on."""
    import torch
    Bt = B.to(dtype).clone()
    St = S.to(dtype).contiguous()
    Et = E.to(dtype).contiguous()
    tmp = torch.empty_like(Bt)
    ohm.ohm_smooth(H, 0, Bt, St, Et, lam_dt, 2, tmp)        # warm
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    ohm.ohm_smooth(H, 0, Bt, St, Et, lam_dt, nsweeps, tmp)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / 1e3 / (2 * nsweeps)


def cpu_baseline(cfg, n_sample):
    """The oracle (FP64, V(2,2)-preconditioned BiCGStab to 1e-10) on one CN step
    of the same workload family at n_sample^3 (r = eta_max dt / h^2 = 16.7)."""
    import ohm_inputs as gen
    from oracle import mg, ref
    c = cfg if n_sample == 128 else gen.config_lognormal128(n_sample)
    t0 = time.perf_counter()
    _, hist = mg.cn_step(c["B"], c["eta"], c["spec"].dx0, c["dt"], rtol=1e-10)
    t = time.perf_counter() - t0
    return {"value": n_sample ** 3 / t, "unit": "cells/s", "cores": ref.threads(), "kind": "oracle",
            "sample": f"one CN step of the {n_sample}^3 log-normal workload (eta 4 decades, dt 100x explicit), "
                      f"FP64 V(2,2)-BiCGStab to 1e-10, {len(hist) - 1} iterations, {t:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--cpu-sample", type=int, default=64, help="grid edge of the oracle sample (0: skip)")
    ap.add_argument("--no-mixed", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see the sharding design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import ohm_inputs as gen
    import paper_1009_0798_amd as ohm

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
    # roofline of the dominant kernel: red-black half-sweep on the level-0 blocks
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
                   "cells": cells, "outer": "BiCGStab", "cycle": "V(2,2)",
                   "iterations_per_step": f64["iters"]},
        "roofline": {"kernel": "k_blk_stencil<double, smooth> (one red-black half-sweep, level 0)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "us_per_launch": t_sw * 1e6, "bytes_per_launch": bytes_sw},
    }
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
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
