"""Benchmark of the SMC sweep on one MI355X.

Workload: the 2-D tracking particle filter at scale -- N = 2^22 particles,
T = 200 observations of a seeded synthetic trajectory, FP64 state and
log-weights, systematic resampling when ESS < N/2.  A "step" is one full
iteration of the sweep: fused move + incremental weight, normalisation (ESS,
log Z, decision), resampling, monitor.  The value is particle-updates per
second (N x timed steps / timed seconds) with every input resident in HBM.

The JSON line also carries the roofline of the dominant kernel (the fused
move + weight sweep, HBM-bound: its algorithmic bytes per launch over its
average duration from HIP events on the launch stream) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
METRIC = "particle-updates/s"


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=189)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--T", type=int, default=200)
    ap.add_argument("--scheme", default="systematic")
    ap.add_argument("--fp32-state", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample-T", type=int, default=30)
    ap.add_argument("--variants", action="store_true",
                    help="also time the FP32-state and multinomial variants")
    return ap.parse_args()


def _bytes_per_particle(fp32: bool, gathered: bool) -> int:
    # state rows in + out, log-weight in + out, ancestor index when gathering
    s = 4 if fp32 else 8
    return 2 * 4 * s + 2 * 8 + (4 if gathered else 0)


def run_pf(args, n, fp32, scheme, steps, warmup, timing=True):
    import torch
    import synth
    from paper_1306_5583_amd import ParticleFilter, _lib as L

    T_needed = 1 + warmup + steps
    T = max(args.T, T_needed)
    _, y = synth.pf_trajectory(T, synth.DATA_SEED[1])
    pf = ParticleFilter(n, y, seed=1, scheme=scheme, fp32_state=fp32)
    stream = pf.stream
    pf.init()
    for t in range(1, 1 + warmup):
        pf.step(t)
    torch.cuda.synchronize()
    m = pf._margs
    if timing:
        # the move kernel of every timed step carries its own start/stop
        # events in its dispatch: no extra packets enter the stream
        L.smc_profile_start(pf.ctx, steps)
    t0 = time.perf_counter()
    for t in range(1 + warmup, 1 + warmup + steps):
        # fused move + weight; the same pass completes the previous step's monitor
        m.obs_index = t
        m.monitor_step = t - 1
        L.smc_move(pf.ctx, t, m)
        L.smc_ess(pf.ctx, t)
        L.smc_resample(pf.ctx, t)
    L.smc_monitor(pf.ctx, warmup + steps)   # the last step's monitor
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    move_ms = L.smc_profile_read(pf.ctx, steps) if timing else []
    pf.check()
    hist = pf.history_host()
    flags = hist[:, L.SMC_H_FLAG]
    tot_bytes = 0.0
    for k, t in enumerate(range(1 + warmup, 1 + warmup + steps)):
        tot_bytes += n * _bytes_per_particle(fp32, bool(flags[t - 1]))
    res = {
        "wall_s": wall,
        "ms_per_step": 1e3 * wall / steps,
        "value": n * steps / wall,
        "move_ms_avg": float(np.mean(move_ms)) if move_ms else None,
        "move_bytes_avg": tot_bytes / max(steps, 1),
        "resample_fraction": float(np.mean(flags[1 + warmup:1 + warmup + steps])),
        "log_z": float(hist[warmup + steps, L.SMC_H_LOGZ]),
    }
    pf.close()
    del pf
    torch.cuda.empty_cache()
    return res


def cpu_baseline(args):
    import oracle
    import synth
    n, T = args.cpu_sample_n, args.cpu_sample_T
    _, y = synth.pf_trajectory(T, synth.DATA_SEED[1])
    cfg = oracle.pf_cfg(n, 1, scheme=args.scheme, fp32_state=args.fp32_state)
    oracle.build()
    t0 = time.perf_counter()
    oracle.pf_run(cfg, y)
    wall = time.perf_counter() - t0
    return {"value": n * T / wall, "unit": METRIC, "cores": 1, "kind": "oracle",
            "sample": "tracking filter, N=%d, %d observations (init + %d steps), %s, "
                      "single-threaded C oracle; wall %.2f s" % (n, T, T - 1, args.scheme, wall)}


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); "
              "multi-GPU sharding is described in DESIGN.md but not implemented" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    n = args.n
    main_res = run_pf(args, n, args.fp32_state, args.scheme, args.steps, args.warmup)
    achieved = main_res["move_bytes_avg"] / (main_res["move_ms_avg"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": METRIC,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-state/f64-weights" if args.fp32_state else "f64",
        "data": "synthetic",
        "config": {"workload": "tracking particle filter (constant-velocity model, Student-t "
                               "observations), N=%d, T=%d, %s, %s resampling at ESS<N/2, "
                               "monitor every step" % (n, max(args.T, 1 + args.warmup + args.steps),
                                                       "fp32 state" if args.fp32_state else "fp64",
                                                       args.scheme),
                   "n": n, "T": max(args.T, 1 + args.warmup + args.steps), "scheme": args.scheme},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "pf_move_kernel (fused move + incremental log-weight)",
                     "avg_launch_ms": main_res["move_ms_avg"],
                     "bytes_per_launch": main_res["move_bytes_avg"]},
        "resample_fraction": main_res["resample_fraction"],
        "log_z": main_res["log_z"],
    }
    if args.variants:
        var = {}
        for name, fp32, scheme in [("fp32_state_systematic", True, "systematic"),
                                   ("fp64_multinomial", False, "multinomial")]:
            r = run_pf(args, n, fp32, scheme, min(args.steps, 60), 5)
            var[name] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                         "move_gbs": r["move_bytes_avg"] / (r["move_ms_avg"] * 1e-3) / 1e9}
        out["variants"] = var
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
