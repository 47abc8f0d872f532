"""Benchmark of the SMC sweep on one MI355X.

Default workload (--workload pf): the 2-D tracking particle filter at scale
-- N = 2^22 particles, T = 200 observations of a seeded synthetic
trajectory, FP64 state and log-weights, systematic resampling when
ESS < N/2.  A "step" is one full iteration of the sweep: fused move +
incremental weight, normalisation (ESS, log Z, decision), resampling,
monitor.  The value is particle-updates per second (N x timed steps / timed
seconds) with every input resident in HBM.

The JSON line carries the roofline of the dominant kernel (the fused move +
weight sweep, HBM-bound: its algorithmic bytes per launch over its average
duration, timed by events carried in each launch's own dispatch), the HBM
traffic the rocprofv3 counters measured for it (from the committed counter
summary, when it was taken on the current kernel source), and the CPU
oracle timed on a bounded sample of the same workload.

Other workloads: --workload gmm-c2 / gmm-c3 (the tempered mixture sampler,
FP64 vector-ALU bound), batch (many filters and samplers in one graph per
step), copy (a plain device copy, the calibration kernel for the traffic
counters and a measured HBM ceiling), study (GPU-seconds per log Z estimate
within 0.05 nats, MALA against random-walk moves).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, published
METRIC = "particle-updates/s"
CSRC = os.path.join(ROOT, "paper_1306_5583_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")

# sources whose change invalidates a stored counter measurement
PF_MOVE_SOURCES = ["smc_pf.hip", "smc_tiles.hpp", "smc_device.hpp", "smc_math.hpp",
                   "smc_internal.hpp"]
GMM_BLOCK_SOURCES = ["smc_gmm_impl.hpp", "smc_device.hpp", "smc_math.hpp", "smc_internal.hpp"]


# move / Metropolis launches timed by dispatch-carried events per run
PROFILE_SAMPLE = 24


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="pf",
                    choices=["pf", "pf-c0", "gmm-c2", "gmm-c3", "batch", "models", "copy",
                             "study"])
    ap.add_argument("--steps", type=int, default=189)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--T", type=int, default=200)
    ap.add_argument("--scheme", default="systematic")
    ap.add_argument("--fp32-state", action="store_true")
    ap.add_argument("--move", default=None, help="gmm: rw or mala (default per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=1 << 20)
    ap.add_argument("--cpu-sample-T", type=int, default=30)
    ap.add_argument("--no-variants", action="store_true",
                    help="pf: skip the FP32-state and multinomial forms of the workload")
    ap.add_argument("--tune", action="store_true", help="batch: run the autotuner first")
    ap.add_argument("--model-seeds", type=int, default=4, help="models: seeds per K")
    ap.add_argument("--study-problem", default="c2", choices=["c2", "c3"])
    ap.add_argument("--study-methods", default="mala,rw,rw:0.05")
    ap.add_argument("--study-tol", type=float, default=0.05)
    ap.add_argument("--study-seeds", type=int, default=16)
    ap.add_argument("--study-seed-base", type=int, default=100000,
                    help="study: first sampler seed of a configuration is base + 1000 T")
    ap.add_argument("--study-ref-method", default=None)
    ap.add_argument("--study-ref-log-z", type=float, default=None)
    ap.add_argument("--study-ref-seeds", type=int, default=4)
    ap.add_argument("--study-ref-n", type=int, default=1 << 18)
    ap.add_argument("--study-ref-T", type=int, default=1600)
    ap.add_argument("--study-T", default="50,100,200,400,800")
    ap.add_argument("--study-logn", default="10,11,12,13,14,15,16")
    return ap.parse_args()


def source_digest(names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(CSRC, nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_profile_values(fname):
    """`value key = v` lines of a committed counter summary (None if absent)."""
    path = os.path.join(PROFILES, fname)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("value ") and "=" in line:
                k, v = line[len("value "):].split("=", 1)
                vals[k.strip()] = v.strip()
    return vals


def _bytes_per_particle(fp32: bool, gathered: bool) -> int:
    """Algorithmic bytes of the fused move + weight per particle: state rows
    in and out, the new log-weight out, and either the old log-weight in or,
    right after a resample (the old weights count as zero and are not read),
    the ancestor index."""
    s = 4 if fp32 else 8
    return 2 * 4 * s + 8 + (4 if gathered else 8)


RESAMPLE_BYTES = 12     # per particle when resampling fires: log-weight in, ancestor out
# per 1024-particle tile and step: tile partial (32 B) and monitor partials
# (40 B) written by the move and read by the normalisation, tile offsets of
# the cumulative weights written (8 B) and read by the resampling (16 B)
TILE_BYTES = 32 + 32 + 40 + 40 + 8 + 16


def _step_bytes(n: int, fp32: bool, gathered: bool, resampled: bool) -> float:
    """Algorithmic HBM bytes of one whole step of the sweep: move + weight,
    normalisation, and the resampling when its decision fires."""
    tiles = -(-n // 1024)
    return (n * (_bytes_per_particle(fp32, gathered) + (RESAMPLE_BYTES if resampled else 0))
            + tiles * TILE_BYTES)


def copy_gbs(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy: (read + write bytes) / time, best of reps."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = max(best, 2 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


# ------------------------------------------------------------ particle filter

def run_pf(args, n, fp32, scheme, steps, warmup, timing=True):
    """Times `steps` whole steps of the filter (wall clock, no events in the
    stream), then, on a second filter of the same size, times the move
    kernel of PROFILE_SAMPLE further steps by events carried in each
    launch's own dispatch (separately, so they cannot slow the timed run)."""
    import torch
    import synth
    from paper_1306_5583_amd import ParticleFilter, _lib as L

    T_needed = 1 + warmup + max(steps, PROFILE_SAMPLE)
    T = max(args.T, T_needed)
    _, y = synth.pf_trajectory(T, synth.DATA_SEED[1])
    # throwaway runs of the same filter first, for at least 0.3 s: the GPU
    # leaves its idle clock state before anything is timed (a few untimed
    # steps are not enough)
    pfw = ParticleFilter(n, y, seed=2, scheme=scheme, fp32_state=fp32)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:
        pfw.run()
        torch.cuda.synchronize()
    pfw.close()
    del pfw

    def issue(pf, t):
        # fused move + weight; the same pass completes the previous step's monitor
        m = pf._margs
        m.obs_index = t
        m.monitor_step = t - 1
        L.smc_move(pf.ctx, t, m)
        L.smc_ess(pf.ctx, t)
        L.smc_resample(pf.ctx, t)

    pf = ParticleFilter(n, y, seed=1, scheme=scheme, fp32_state=fp32)
    pf.init()
    for t in range(1, 1 + warmup):
        issue(pf, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1 + warmup, 1 + warmup + steps):
        issue(pf, t)
    L.smc_monitor(pf.ctx, warmup + steps)   # the last step's monitor
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pf.check()
    hist = pf.history_host()
    flags = hist[:, L.SMC_H_FLAG]
    step_bytes = [_step_bytes(n, fp32, bool(flags[t - 1]), bool(flags[t]))
                  for t in range(1 + warmup, 1 + warmup + steps)]
    res = {
        "wall_s": wall,
        "ms_per_step": 1e3 * wall / steps,
        "value": n * steps / wall,
        "step_bytes_avg": float(np.mean(step_bytes)),
        "resample_fraction": float(np.mean(flags[1 + warmup:1 + warmup + steps])),
        "log_z": float(hist[warmup + steps, L.SMC_H_LOGZ]),
    }
    pf.close()
    del pf
    if timing:
        pf = ParticleFilter(n, y, seed=1, scheme=scheme, fp32_state=fp32)
        pf.init()
        for t in range(1, 1 + warmup):
            issue(pf, t)
        sample = PROFILE_SAMPLE
        L.smc_profile_start(pf.ctx, sample)
        for t in range(1 + warmup, 1 + warmup + sample):
            issue(pf, t)
        torch.cuda.synchronize()
        move_ms = L.smc_profile_read(pf.ctx, sample)
        pf.check()
        flags = pf.history_host()[:, L.SMC_H_FLAG]
        res["move_ms_avg"] = float(np.mean(move_ms))
        res["move_bytes_avg"] = float(np.mean(
            [n * _bytes_per_particle(fp32, bool(flags[t - 1]))
             for t in range(1 + warmup, 1 + warmup + sample)]))
        pf.close()
        del pf
    torch.cuda.empty_cache()
    return res


def _cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _host_threads():
    """Threads for the all-core oracle timing: the CPU share of this process
    (its affinity mask), at most 16 (the host cores one GPU is given)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline_pf(args, fp32=False, scheme=None):
    """The oracle on the host of the GPU machine, on bounded samples of the workload (the
    first 30 observations): all the process's cores (up to 16) at the full
    particle count, and one thread at N = 2^20.  The oracle runs its
    per-particle loops on the threads and its sums sequentially, so both
    give the results of the sequential oracle."""
    import oracle
    import synth
    scheme = scheme or args.scheme
    oracle.build()
    out = {}
    threads = _host_threads()
    for label, th, n, T in (("one_thread", 1, args.cpu_sample_n, args.cpu_sample_T),
                            ("all_cores", threads, args.n, args.cpu_sample_T)):
        _, y = synth.pf_trajectory(T, synth.DATA_SEED[1])
        cfg = oracle.pf_cfg(n, 1, scheme=scheme, fp32_state=fp32)
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.pf_run(cfg, y)
        wall = time.perf_counter() - t0
        out[label] = {"value": n * (T - 1) / wall, "cores": th, "n": n, "T": T, "wall_s": wall}
    oracle.set_threads(threads)
    best = out["all_cores"]
    res = {"value": best["value"], "unit": METRIC, "cores": best["cores"], "kind": "oracle",
           "sample": "tracking filter at the full particle count, the first observations "
                     "(N=%d, %d observations: init + %d steps, init inside the wall), %s%s, C "
                     "oracle with its per-particle loops on %d threads (sums sequential); "
                     "wall %.1f s"
                     % (best["n"], best["T"], best["T"] - 1, scheme,
                        ", fp32 state" if fp32 else "", best["cores"], best["wall_s"]),
           "one_thread": dict(out["one_thread"], unit=METRIC,
                              sample="N=%d, %d observations, 1 thread"
                                     % (out["one_thread"]["n"], out["one_thread"]["T"]))}
    res.update(_cpu_info())
    return res


def cpu_baseline_gmm(workload, K, nd, y, move):
    """The oracle's whole sampler (Algorithm 'gmm', same data, schedule and
    move) on bounded samples: fewer particles and the first steps of the
    schedule (the work per step does not depend on alpha); one thread, and
    all the process's cores (up to 16) on a sample four times as large."""
    import oracle
    import synth
    from paper_1306_5583_amd import mala_scales, rw_scales
    n1, Ts, T = (1 << 12, 25, 100) if workload == "gmm-c2" else (1 << 9, 10, 200)
    alphas = synth.prior_tempering(T, 4.0)[:Ts + 1]
    f = rw_scales if move == "rw" else mala_scales
    scales = np.array([f(a) for a in alphas])
    oracle.build()
    threads = _host_threads()
    out = {}
    for label, th, n in (("one_thread", 1, n1), ("all_cores", threads, 4 * n1)):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        oracle.gmm_run(oracle.gmm_cfg(n, 1, K, move=move), y, alphas, scales)
        wall = time.perf_counter() - t0
        out[label] = {"value": n * Ts / wall, "cores": th, "n": n, "steps": Ts, "wall_s": wall}
    oracle.set_threads(threads)
    best = out["all_cores"]
    res = {"value": best["value"], "unit": METRIC, "cores": best["cores"], "kind": "oracle",
           "sample": "mixture sampler K=%d, n=%d data, N=%d, the first %d of %d steps (init "
                     "inside the wall), %s moves, C oracle with its per-particle loops on %d "
                     "threads (sums sequential); wall %.2f s"
                     % (K, nd, best["n"], Ts, T, move, best["cores"], best["wall_s"]),
           "one_thread": dict(out["one_thread"], unit=METRIC,
                              sample="N=%d, first %d steps, 1 thread"
                                     % (out["one_thread"]["n"], Ts))}
    res.update(_cpu_info())
    return res


def pf_traffic():
    """HBM bytes per move launch from the committed FETCH_SIZE / WRITE_SIZE
    summary, scaled by the copy-kernel calibration; None when the summary
    was taken on another version of the kernel."""
    v = read_profile_values("pf_move_c1_traffic.txt")
    if not v or v.get("source_digest") != source_digest(PF_MOVE_SOURCES):
        return None
    fetch = float(v["fetch_kib_per_launch"]) * 1024 / float(v["copy_fetch_factor"])
    write = float(v["write_kib_per_launch"]) * 1024 / float(v["copy_write_factor"])
    return fetch + write


def _pf_label(fp32, scheme):
    return "%s_%s" % ("fp32_state" if fp32 else "fp64", scheme)


def _sweep(res):
    """Whole-step HBM figures: algorithmic bytes of the step (move + weight,
    normalisation, resampling when it fired) over the wall time per step."""
    gbs = res["step_bytes_avg"] / (res["ms_per_step"] * 1e-3) / 1e9
    return {"bytes_per_step": res["step_bytes_avg"], "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def bench_pf(args):
    n = args.n
    main_res = run_pf(args, n, args.fp32_state, args.scheme, args.steps, args.warmup)
    achieved = main_res["move_bytes_avg"] / (main_res["move_ms_avg"] * 1e-3) / 1e9
    traffic = None
    if not args.fp32_state and n == 1 << 22 and args.scheme == "systematic":
        traffic = pf_traffic()
    T = max(args.T, 1 + args.warmup + args.steps)
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
                               "monitor every step" % (n, T, "fp32 state" if args.fp32_state
                                                       else "fp64", args.scheme),
                   "n": n, "T": T, "scheme": args.scheme},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "pf_move_kernel (fused move + incremental log-weight)",
                     "avg_launch_ms": main_res["move_ms_avg"],
                     "bytes_per_launch": main_res["move_bytes_avg"],
                     "timing": "events in the dispatch of %d move launches of a separate run "
                               "after the timed steps" % PROFILE_SAMPLE},
        "sweep_roofline": _sweep(main_res),
        "resample_fraction": main_res["resample_fraction"],
        "log_z": main_res["log_z"],
        "hbm_copy_gbs": copy_gbs(),
    }
    if not args.no_variants:
        # the rest of the workload's four forms: {fp64, fp32 state} x
        # {systematic, multinomial}
        var = {}
        for fp32 in (False, True):
            for scheme in ("systematic", "multinomial"):
                if fp32 == args.fp32_state and scheme == args.scheme:
                    continue
                r = run_pf(args, n, fp32, scheme, min(args.steps, 60), 5)
                mg = r["move_bytes_avg"] / (r["move_ms_avg"] * 1e-3) / 1e9
                var[_pf_label(fp32, scheme)] = {
                    "value": r["value"], "ms_per_step": r["ms_per_step"],
                    "steps": min(args.steps, 60),
                    "resample_fraction": r["resample_fraction"],
                    "sweep_roofline": _sweep(r),
                    "move_kernel": {"achieved": mg, "frac": mg / HBM_PEAK_GBS,
                                    "avg_launch_ms": r["move_ms_avg"],
                                    "bytes_per_launch": r["move_bytes_avg"]}}
        out["variants"] = var
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_pf(args, args.fp32_state, args.scheme)
    return out


def bench_pf_c0(args):
    """The small filter (N = 1000, T = 100): launch-latency bound, so the
    run is timed three ways: eagerly (three launches per step from the
    host), as the whole run captured in one graph and replayed, and as the
    batched form with one problem (one persistent launch per step, a graph
    replay per step)."""
    import torch
    import synth
    import paper_1306_5583_amd as pkg
    _, y = synth.pf_trajectory(100, synth.DATA_SEED[0])
    steps = y.shape[0] - 1
    reps = 5
    pf = pkg.ParticleFilter(1000, y, seed=1)
    pf.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        logz_eager = pf.run()
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / (reps * steps)
    # the same runs (prior draws, every step, the last monitor) as one graph
    g = pf.capture_run()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    run_graph_ms = 1e3 * (time.perf_counter() - t0) / (reps * steps)
    logz_run_graph = pf.log_z()
    pf.close()
    br = pkg.BatchRunner([pkg.PfSpec(n=1000, y=y, seed=1)])
    br.run(steps, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = np.array(br.run(steps, graph=True, latencies=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    logz_graph = br.log_z(0)
    br.close()
    # the value is the fastest of the three ways of issuing the same steps;
    # all are reported
    forms = {"eager launches": eager_ms * 1e-3 * steps,
             "whole run as one graph": run_graph_ms * 1e-3 * steps,
             "one persistent launch per step, graph replay per step": wall}
    best = min(forms, key=forms.get)
    best_wall = forms[best]
    return {
        "metric": METRIC, "value": 1000 * steps / best_wall, "unit": METRIC, "n_gpus": 1,
        "steps": steps, "warmup": 1, "ms_per_step": 1e3 * best_wall / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tracking particle filter, N=1000, T=100, systematic at "
                               "ESS<N/2, %s" % best,
                   "n": 1000, "T": 100},
        "latency_ms": {"graph_p50": float(np.percentile(lat, 50)),
                       "graph_p99": float(np.percentile(lat, 99)),
                       "eager_mean": eager_ms, "run_graph_mean": run_graph_ms},
        "log_z": {"eager": logz_eager, "run_graph": logz_run_graph, "graph": logz_graph},
    }


# ------------------------------------------------------------ mixture sampler

def gmm_config(which, move):
    import synth
    if which == "gmm-c2":
        K, n, nd, T = 4, 1 << 14, 1000, 100
        y = synth.gmm_data_four_components(nd, synth.DATA_SEED[2])
        move = move or "rw"
    else:
        K, n, nd, T = 6, 1 << 16, 10000, 200
        y, _ = synth.gmm_data_spaced(nd, K, synth.DATA_SEED[3])
        move = move or "mala"
    return K, n, nd, T, y, move


def bench_gmm(args):
    import torch
    import synth
    from paper_1306_5583_amd import GmmSampler, _lib as L
    K, n, nd, T, y, move = gmm_config(args.workload, args.move)
    alphas = synth.prior_tempering(T, 4.0)
    # throwaway runs first, for at least 0.3 s (the GPU leaves its idle clock
    # state; one short run of the small workload is not enough)
    warm = GmmSampler(n, y, K, T, seed=2, move=move)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:
        warm.run(alphas[:min(T, 40) + 1])
        torch.cuda.synchronize()
    warm.close()
    s = GmmSampler(n, y, K, T, seed=1, move=move)
    blocks = 3 if K > 1 else 2
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    logz = s.run(alphas)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.check()
    # one Metropolis launch per step covers its `blocks` likelihood passes;
    # PROFILE_SAMPLE of them are timed by events in their own dispatch, in a
    # separate run after the timed one
    sample = min(T, PROFILE_SAMPLE)
    p = GmmSampler(n, y, K, T, seed=3, move=move)
    L.smc_profile_start(p.ctx, sample)
    p.run(alphas[:sample + 1])
    torch.cuda.synchronize()
    blk_ms = L.smc_profile_read(p.ctx, sample)
    p.check()
    p.close()
    hist = s.history_host()
    terms_per_launch = n * nd * K * blocks
    avg_ms = float(np.mean(blk_ms))
    v = read_profile_values("gmm_block_%s_fp64.txt" % args.workload.split("-")[1])
    flops = None
    if v and v.get("source_digest") == source_digest(GMM_BLOCK_SOURCES) \
            and v.get("move") == move:
        flops = float(v["fp64_flops_per_term"]) * terms_per_launch
    achieved = flops / (avg_ms * 1e-3) / 1e12 if flops else None
    out = {
        "metric": METRIC, "value": n * T / wall, "unit": METRIC, "n_gpus": 1, "steps": T,
        "warmup": 3, "ms_per_step": 1e3 * wall / T, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "tempered Gaussian-mixture SMC sampler, K=%d, n=%d data, N=%d, "
                               "T=%d, alpha=(t/T)^4, %s moves" % (K, nd, n, T, move),
                   "K": K, "n_data": nd, "n": n, "T": T, "move": move},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                     "traffic": None, "kernel": "gmm_step_kernel (the step's Metropolis blocks: "
                     "proposal, mixture likelihood%s, accept)" % (" and gradient" if move == "mala"
                                                                 else ""),
                     "avg_launch_ms": avg_ms, "terms_per_launch": terms_per_launch},
        "terms_per_s": terms_per_launch / (avg_ms * 1e-3),
        "log_z": logz,
        "log_z_path_sampling": s.log_z_path(),
        "accept_rate": (hist[1:, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3].sum(axis=0) / (n * T)).tolist(),
        "resamples": int(hist[1:, L.SMC_H_FLAG].sum()),
    }
    s.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_gmm(args.workload, K, nd, y, move)
    return out


# ------------------------------------------------------------ batched form

def bench_batch(args):
    import torch
    import synth
    import paper_1306_5583_amd as pkg
    steps = 200
    work = synth.batched_workload(steps)
    specs = [pkg.PfSpec(**kw) if k == "pf" else pkg.GmmSpec(move="mala", **kw)
             for k, kw in work]
    br = pkg.BatchRunner(specs)
    if args.tune:
        br.autotune(3, None)
    br.run(3, graph=True)          # warm-up (graph capture included)
    br.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = np.array(br.run(steps, graph=True, latencies=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    br.check()
    parts = sum(int(kw["n"]) for _, kw in work)
    out = {
        "metric": METRIC, "value": parts * steps / wall, "unit": METRIC, "n_gpus": 1,
        "steps": steps, "warmup": 3, "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched: 128 tracking filters (N log-uniform in [2^10, 2^18]) "
                               "+ 32 MALA mixture samplers (K in 2..8, n log-uniform in "
                               "[500, 20000], N log-uniform in [2^12, 2^16]), 200 steps, each "
                               "step one persistent launch (captured in a HIP graph)",
                   "problems": len(work), "particles": parts},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "schedule": br.schedule(),
        "tuned": bool(args.tune),
    }
    br.close()
    return out


# ------------------------------------------- model comparison over K (batched)

def bench_models(args):
    """Bayesian model comparison over the number of mixture components
    (Section 5.2: the evidence p(y | M_r) of every r = 1..8 on the
    four-component data of the random-walk sampler, several seeds each),
    all samplers advanced together, one persistent launch per step.
    Posterior model probabilities assume a uniform prior over r."""
    import torch
    import synth
    import paper_1306_5583_amd as pkg
    y = synth.gmm_data_four_components(1000, synth.DATA_SEED[2])
    T, n = 100, 1 << 14
    alphas = synth.prior_tempering(T, 4.0)
    Ks = list(range(1, 9))
    seeds = list(range(1, args.model_seeds + 1))
    specs = [pkg.GmmSpec(n=n, y=y, K=K, alphas=alphas, move="rw", seed=s,
                         problem_id=100 * K + s) for K in Ks for s in seeds]
    br = pkg.BatchRunner(specs)
    br.run(2, graph=True)          # warm-up (graph capture included)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = np.array(br.run(T, graph=True, latencies=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    br.check()
    logz = np.array([br.log_z(i) for i in range(len(specs))]).reshape(len(Ks), len(seeds))
    mean = logz.mean(axis=1)
    se = logz.std(axis=1, ddof=1) / np.sqrt(len(seeds)) if len(seeds) > 1 else np.zeros(len(Ks))
    post = np.exp(mean - mean.max())
    post /= post.sum()
    br.close()
    parts = n * len(specs)
    return {
        "metric": METRIC, "value": parts * T / wall, "unit": METRIC, "n_gpus": 1,
        "steps": T, "warmup": 2, "ms_per_step": 1e3 * wall / T, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "model comparison: random-walk mixture samplers for K=1..8 "
                               "(x%d seeds), n=1000 four-component data, N=2^14 each, T=100, "
                               "alpha=(t/T)^4, one persistent launch per step" % len(seeds),
                   "K": Ks, "seeds": len(seeds), "n": n, "T": T},
        "log_z": {str(K): float(m) for K, m in zip(Ks, mean)},
        "log_z_se": {str(K): float(e) for K, e in zip(Ks, se)},
        "posterior_K": {str(K): float(p) for K, p in zip(Ks, post)},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
    }


# ------------------------------------------------- MALA vs random walk study

def _method_scales(method, alphas):
    """'mala' / 'mala:h' (MALA step h, default 0.05; 'malaad:h' the same
    steps times per-block factors that follow the acceptance rates, see
    BlockAdapter), 'rw' / 'rw:b' ('rwad:b' acceptance-adapted) (random
    walk with the paper's alpha-adaptive per-block scales rescaled to base b,
    default 0.15) or 'rwfixed:s' (random walk with the same standard
    deviation s in every block and step): the move kind and the per-step
    block scales."""
    from paper_1306_5583_amd import mala_scales, rw_scales
    kind, _, par = method.partition(":")
    if kind in ("mala", "malaad"):
        h = float(par) if par else 0.05
        return "mala", np.array([mala_scales(min(max(a, 0.0), 1.0), h) for a in alphas])
    if kind == "rwfixed":
        sd = float(par) if par else 0.15
        return "rw", np.full((len(alphas), 3), sd)
    b = float(par) if par else 0.15  # 'rw' and 'rwad' (the same, acceptance-adapted)
    return "rw", np.array([rw_scales(min(max(a, 0.0), 1.0), b) for a in alphas])


def _study_batch(y, K, n, T, method, seeds, seed0):
    """`seeds` independent samplers of one configuration in one batch;
    returns (log Z estimates, wall seconds of init + T graph replays)."""
    import torch
    import synth
    import paper_1306_5583_amd as pkg
    alphas = synth.prior_tempering(T, 4.0)
    move, scales = _method_scales(method, alphas)
    specs = [pkg.GmmSpec(n=n, y=y, K=K, alphas=alphas, scales=scales, move=move,
                         seed=seed0 + s, problem_id=s) for s in range(seeds)]
    br = pkg.BatchRunner(specs)
    adapt = method.startswith(("malaad", "rwad"))
    ads = [pkg.BlockAdapter(move) for _ in range(seeds)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    br.init()
    br.capture()
    for k in range(T):
        br.replay()
        if adapt and k + 1 < T:
            # each sampler's block scales follow its acceptance rates
            # (BlockAdapter: towards 0.574 for MALA, 0.234 for the random walk)
            acc = br.accept_counts(k + 1)
            for s in range(seeds):
                br.set_block_scales(s, k + 2, scales[k + 2] * ads[s].update(acc[s], n))
        if (k + 1) % 200 == 0 and k + 1 < T:
            # a progress line per 200 steps (long configurations run for minutes)
            br.stream.synchronize()
            print("#   %s N=%d T=%d: step %d, %.1f s" % (method, n, T, k + 1,
                                                        time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    br.check()
    z = [br.log_z(i) for i in range(seeds)]
    br.close()
    return np.array(z), wall


def bench_study(args):
    """GPU-seconds per log Z estimate within 0.05 nats (root-mean-square over
    seeds, against a high-effort reference run with the first method) for
    MALA and random-walk moves.  Each configuration runs its seeds as one
    batch; the cost of one estimate is the batch wall time over the seed
    count."""
    K, _, nd, _, y, _ = gmm_config("gmm-" + args.study_problem, None)
    methods = args.study_methods.split(",")
    ref_method = args.study_ref_method or methods[0]
    if args.study_ref_log_z is not None:
        zstar = args.study_ref_log_z
        ref = {"log_z_given": zstar}
    else:
        zr, wall = _study_batch(y, K, args.study_ref_n, args.study_ref_T, ref_method,
                                args.study_ref_seeds, 7000)
        zstar = float(zr.mean())
        ref = {"method": ref_method, "n": args.study_ref_n, "T": args.study_ref_T,
               "log_z": zr.tolist(), "mean": zstar,
               "se": float(zr.std(ddof=1) / np.sqrt(zr.size)), "wall_s": wall}
        print("# reference %s N=%d T=%d: %s (%.1f s)" % (ref_method, args.study_ref_n,
                                                       args.study_ref_T,
                                                       np.round(zr, 4).tolist(), wall),
              file=sys.stderr, flush=True)
    Ts = [int(v) for v in args.study_T.split(",")]
    Ns = [1 << int(v) for v in args.study_logn.split(",")]
    grid = []
    best = {}
    for method in methods:
        for T in Ts:
            for n in Ns:
                z, wall = _study_batch(y, K, n, T, method, args.study_seeds,
                                       args.study_seed_base + 1000 * T)
                rmse = float(np.sqrt(np.mean((z - zstar) ** 2)))
                cost = wall / args.study_seeds
                grid.append({"method": method, "T": T, "n": n, "rmse": rmse,
                             "bias": float(z.mean() - zstar), "sd": float(z.std(ddof=1)),
                             "gpu_s": cost, "log_z": z.tolist()})
                print("# %s T=%d N=%d rmse %.4f bias %+.4f sd %.4f gpu_s %.4f" % (
                    method, T, n, rmse, z.mean() - zstar, z.std(ddof=1), cost),
                    file=sys.stderr, flush=True)
                if rmse <= args.study_tol and (method not in best
                                               or cost < best[method]["gpu_s"]):
                    best[method] = {"T": T, "n": n, "rmse": rmse, "gpu_s": cost}
    rw_best = [b["gpu_s"] for m, b in best.items() if m.startswith("rw")]
    mala_best = [b["gpu_s"] for m, b in best.items() if m.startswith("mala")]
    out = {
        "metric": "GMM-SMC GPU-s to +-%g nats log Z, MALA vs RW" % args.study_tol,
        "workload": "tempered Gaussian-mixture sampler, %s data: K=%d, n=%d, alpha=(t/T)^4"
                    % (args.study_problem, K, nd),
        "reference": ref,
        "tolerance_nats": args.study_tol,
        "best": best,
        "mala_over_best_rw_cost": (min(mala_best) / min(rw_best)
                                   if mala_best and rw_best else None),
        "seeds": args.study_seeds,
        "grid": grid,
    }
    return out


def bench_copy(args):
    nbytes = 1 << 30
    return {"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
            "gbs": copy_gbs(nbytes)}


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus %d requested); the sweep is not sharded "
              "across GPUs" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "pf":
        out = bench_pf(args)
    elif args.workload == "pf-c0":
        out = bench_pf_c0(args)
    elif args.workload in ("gmm-c2", "gmm-c3"):
        out = bench_gmm(args)
    elif args.workload == "batch":
        out = bench_batch(args)
    elif args.workload == "models":
        out = bench_models(args)
    elif args.workload == "study":
        out = bench_study(args)
    else:
        out = bench_copy(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
