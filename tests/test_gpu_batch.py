"""Batched form: many filters and samplers of uneven sizes in one launch per
phase.  Each problem must be its own single-problem algorithm with its
problem id in the Philox counter, so the batch is checked (a) against the
oracle run of each problem, (b) against the single-problem GPU path and
(c) between eager steps and graph replays."""
import math
import os

import numpy as np
import pytest

import synth
from gpu_helpers import assert_close_l1, assert_gmm_run_matches

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_5583_amd as pkg
    from paper_1306_5583_amd import _lib as L
    return pkg, L


def _say(*a):
    print("[batch]", *a, flush=True)


def _small_workload(steps):
    """Ragged sizes spanning several tiles; K = 1 included."""
    rng = np.random.default_rng(41)
    probs = []
    for n in (1000, 3001, 5120):
        probs.append(synth.BatchProblem("pf", n, int(rng.integers(1, 1 << 40)),
                                        int(rng.integers(1, 1000))))
    for n, K, nd in ((2048, 3, 90), (1500, 1, 60), (3333, 5, 130), (700, 2, 45)):
        probs.append(synth.BatchProblem("gmm", n, int(rng.integers(1, 1 << 40)),
                                        int(rng.integers(1, 1000)), K, nd))
    return synth.batched_workload(steps, probs)


def _specs(pkg, work, move="mala"):
    out = []
    for kind, kw in work:
        if kind == "pf":
            out.append(pkg.PfSpec(**kw))
        else:
            out.append(pkg.GmmSpec(move=move, **kw))
    return out


def _orc_cfg(orc, kind, kw, move):
    if kind == "pf":
        return orc.pf_cfg(kw["n"], kw["seed"], problem=kw["problem_id"])
    return orc.gmm_cfg(kw["n"], kw["seed"], kw["K"], problem=kw["problem_id"], move=move)


@pytest.mark.parametrize("move", ["mala", "rw"])
def test_batch_matches_oracle(lib, orc, move):
    pkg, L = lib
    steps = 10
    work = _small_workload(steps)
    specs = _specs(pkg, work, move)
    _say("oracle parity", move, [(k, kw["n"]) for k, kw in work])
    br = pkg.BatchRunner(specs)
    br.run(steps, graph=True)
    br.check()
    for i, (kind, kw) in enumerate(work):
        h = br.history_host(i)
        cfg = _orc_cfg(orc, kind, kw, move)
        if kind == "pf":
            logz_o, hist_o, xf_o, _ = orc.pf_run(cfg, kw["y"])
            scale = max(1.0, np.abs(hist_o[:, 2]).sum())
            assert abs(br.log_z(i) - logz_o) <= 1e-12 * scale, (i, br.log_z(i), logz_o)
            assert np.array_equal(h[:steps + 1, L.SMC_H_FLAG], hist_o[:, 1])
            assert_close_l1(h[:steps + 1, L.SMC_H_ESS], hist_o[:, 0], hist_o[:, 0], 1e-11, "ess")
            # the monitor of step t is completed by step t + 1's pass
            assert_close_l1(h[:steps, L.SMC_H_MON:L.SMC_H_MON + 4], hist_o[:steps, 5:9], 20.0,
                            1e-11, "means")
            x = br.state(i).cpu().numpy()[:4]
            if h[steps, L.SMC_H_FLAG] == 1:  # ancestors still pending
                x = x[:, br.bufs[i].ancestors.cpu().numpy()]
            assert_close_l1(x, xf_o, np.abs(xf_o) + 1.0, 1e-11, "state")
        else:
            sched = pkg.batch.gmm_schedule(kw["alphas"], None, move)
            logz_o, hist_o, pop_o, _ = orc.gmm_run(cfg, kw["y"], sched[:, 0], sched[:, 1:])
            # exact decisions and 1e-12 agreement (the path-sampling U_t and
            # trapezoid included) up to the first step whose decisions the
            # oracle records inside a boundary window
            ts = assert_gmm_run_matches(h[:steps + 1], hist_o, sched[:, 0], L,
                                        "problem %d" % i)
            assert br.log_z_path(i) == h[steps, L.SMC_H_PS]
            assert ts == steps + 1, (i, ts)
            D = 3 * kw["K"] - 1
            st = br.state(i).cpu().numpy()[:D]
            assert_close_l1(st, pop_o, np.abs(pop_o) + 1.0, 1e-12, "problem %d population" % i)


def test_batch_equals_single_problem_runs(lib, orc):
    pkg, L = lib
    steps = 8
    work = _small_workload(steps)
    br = pkg.BatchRunner(_specs(pkg, work))
    br.run(steps, graph=False)
    br.check()
    for i, (kind, kw) in enumerate(work):
        h = br.history_host(i)
        if kind == "pf":
            pf = pkg.ParticleFilter(kw["n"], kw["y"], seed=kw["seed"], problem_id=kw["problem_id"])
            pf.run()
            hs = pf.history_host()
            # same kernels, same tiles: identical bits
            cols = [L.SMC_H_ESS, L.SMC_H_FLAG, L.SMC_H_DLOGZ, L.SMC_H_LOGZ, L.SMC_H_L]
            assert np.array_equal(h[:, cols], hs[:, cols]), i
            assert np.array_equal(br.state(i).cpu().numpy(), pf.state().cpu().numpy()), i
        else:
            s = pkg.GmmSampler(kw["n"], kw["y"], kw["K"], steps, seed=kw["seed"],
                               problem_id=kw["problem_id"], move="mala")
            s.run(kw["alphas"])
            hs = s.history_host()
            # the waves per tile may differ, so the likelihood sums in another
            # order: identical decisions, and 1e-12 agreement, wherever the
            # oracle records no decision inside a boundary window
            sched = pkg.batch.gmm_schedule(kw["alphas"], None, "mala")
            _, hist_o, _, _ = orc.gmm_run(_orc_cfg(orc, kind, kw, "mala"), kw["y"], sched[:, 0],
                                          sched[:, 1:])
            ts = assert_gmm_run_matches(h[:steps + 1], hist_o, sched[:, 0], L,
                                        "batch problem %d" % i)
            assert ts == steps + 1, (i, ts)
            assert_gmm_run_matches(hs[:steps + 1], hist_o, sched[:, 0], L,
                                   "single problem %d" % i)


def test_graph_replays_equal_eager_steps(lib):
    pkg, L = lib
    steps = 6
    work = _small_workload(steps)
    a = pkg.BatchRunner(_specs(pkg, work))
    a.run(steps, graph=False)
    b = pkg.BatchRunner(_specs(pkg, work))
    b.run(steps, graph=True)
    a.check()
    b.check()
    for i in range(len(work)):
        assert np.array_equal(a.history_host(i), b.history_host(i)), i
        assert np.array_equal(a.state(i).cpu().numpy(), b.state(i).cpu().numpy()), i
    # a second run on the same buffers (init again, replay the same graph)
    b.init()
    for _ in range(steps):
        b.replay()
    b.check()
    for i in range(len(work)):
        assert np.array_equal(a.history_host(i), b.history_host(i)), i


def test_step_limits_and_order(lib):
    pkg, L = lib
    work = _small_workload(3)
    br = pkg.BatchRunner(_specs(pkg, work))
    with pytest.raises(pkg.SmcError):
        br.step()  # before init
    with pytest.raises(pkg.SmcError):
        br.replay()  # before capture
    br.init()
    for _ in range(3):
        br.step()
    with pytest.raises(pkg.SmcError):
        br.step()  # schedules / observations exhausted
    br.check()


def test_autotune_and_cache(lib, tmp_path):
    # the tuner times whole steps for every schedule candidate; a schedule
    # only changes which workgroup takes which item, never the arithmetic,
    # so the tuned run is bit-identical to the default one
    pkg, L = lib
    steps = 5
    work = _small_workload(steps)
    cache = str(tmp_path / "tune.txt")
    br = pkg.BatchRunner(_specs(pkg, work))
    ref = pkg.BatchRunner(_specs(pkg, work))
    ref.run(steps, graph=True)
    br.autotune(repeats=3, cache_path=cache)
    sch = br.schedule()
    _say("tuned schedule", sch)
    assert sch["order"] in (0, 1) and sch["per_item"] in (1, 2) and sch["wgs_per_cu"] >= 1
    # the grid: workgroups per compute unit times the compute units, but no
    # more workgroups than the step has items
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert sch["workgroups"] == min(sch["wgs_per_cu"] * cus, sch["items"]), (sch, cus)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and "order=%d per_item=%d wgs_per_cu=%d" % (
        sch["order"], sch["per_item"], sch["wgs_per_cu"]) in lines[0]
    br.run(steps, graph=True)
    br.check()
    for i in range(len(work)):
        assert np.array_equal(br.history_host(i), ref.history_host(i)), i
        assert np.array_equal(br.state(i).cpu().numpy(), ref.state(i).cpu().numpy()), i
    # a second tuner call reads the cache and does not append
    br2 = pkg.BatchRunner(_specs(pkg, work))
    br2.autotune(repeats=3, cache_path=cache)
    assert br2.schedule() == sch
    assert open(cache).read().strip().splitlines() == lines


def test_every_schedule_gives_the_same_bits(lib):
    # queue orders, tiles per Metropolis item and workgroup counts: the
    # dependency waits make every schedule compute the same thing
    pkg, L = lib
    steps = 4
    work = _small_workload(steps)
    ref = None
    for order, per_item, wgs in [(0, 1, 2), (1, 2, 1), (0, 2, 1), (1, 1, 2)]:
        br = pkg.BatchRunner(_specs(pkg, work))
        L.load()
        br.set_schedule(order, per_item, wgs)
        br.run(steps, graph=(order == 0))
        br.check()
        got = [(br.history_host(i).copy(), br.state(i).cpu().numpy().copy())
               for i in range(len(work))]
        _say("schedule", order, per_item, wgs, br.schedule())
        if ref is None:
            ref = got
        else:
            for i, ((h0, x0), (h1, x1)) in enumerate(zip(ref, got)):
                assert np.array_equal(h0, h1), (order, per_item, wgs, i)
                assert np.array_equal(x0, x1), (order, per_item, wgs, i)
        br.close()


def test_schedule_change_mid_run_keeps_the_bits(lib):
    # a new schedule changes the tickets a step consumes; the steps taken
    # before it keep their indices, so the run continues exactly
    pkg, L = lib
    steps = 4
    work = _small_workload(steps)
    ref = pkg.BatchRunner(_specs(pkg, work))
    ref.run(steps, graph=False)
    ref.check()
    want = [(ref.history_host(i).copy(), ref.state(i).cpu().numpy().copy())
            for i in range(len(work))]
    ref.close()
    br = pkg.BatchRunner(_specs(pkg, work))
    br.set_schedule(0, 1, 2)
    br.init()
    br.step()
    br.step()
    br.set_schedule(1, 2, 1)   # other queue order, item size and grid
    _say("schedule after the change", br.schedule())
    br.step()
    br.capture()               # and the rest as graph replays
    br.replay()
    br.check()
    for i, (h0, x0) in enumerate(want):
        assert np.array_equal(h0, br.history_host(i)), i
        assert np.array_equal(x0, br.state(i).cpu().numpy()), i
    br.close()


def test_small_batch_grid_is_capped_at_its_items(lib):
    # one small filter: the launch has no more workgroups than items
    pkg, L = lib
    work = _small_workload(2)
    br = pkg.BatchRunner(_specs(pkg, work[:1]))
    sch = br.schedule()
    assert sch["workgroups"] <= sch["items"], sch
    br.run(2, graph=True)
    br.check()
    br.close()


def test_repeated_runs_are_bit_identical(lib):
    # many small samplers whose normalisation, resampling and Metropolis
    # items follow each other closely on different XCDs: a release that
    # lets a counter overtake its data shows up as runs that differ (a
    # stale tile partial changed L, the ESS and every later step)
    pkg, L = lib
    steps = 60
    rng = np.random.default_rng(909)
    probs = [synth.BatchProblem("gmm", 2048, int(rng.integers(1, 1 << 40)),
                                int(rng.integers(1, 1000)), 3, 120) for _ in range(48)]
    work = synth.batched_workload(steps, probs)
    out = []
    for rep in range(2):
        br = pkg.BatchRunner(_specs(pkg, work))
        br.run(steps, graph=True)
        br.check()
        out.append([br.history_host(i).copy() for i in range(len(work))])
        br.close()
    for i, (h0, h1) in enumerate(zip(*out)):
        assert np.array_equal(h0, h1), i


def test_batch_variants_match_oracle(lib, orc):
    """What the single-problem contexts allow, batched: FP32 filter state,
    stratified resampling for filters and samplers, random-walk and MALA
    samplers in one batch, two Metropolis sweeps."""
    pkg, L = lib
    steps = 8
    rng = np.random.default_rng(77)
    base = [synth.BatchProblem("pf", 3001, 11, 21), synth.BatchProblem("pf", 2048, 12, 22),
            synth.BatchProblem("gmm", 2500, 13, 23, 3, 80), synth.BatchProblem("gmm", 1800, 14, 24, 4, 60),
            synth.BatchProblem("gmm", 1100, 15, 25, 2, 50)]
    work = synth.batched_workload(steps, base)
    specs = [pkg.PfSpec(fp32_state=True, **work[0][1]),
             pkg.PfSpec(scheme="stratified", **work[1][1]),
             pkg.GmmSpec(move="rw", scheme="stratified", **work[2][1]),
             pkg.GmmSpec(move="mala", sweeps=2, **work[3][1]),
             pkg.GmmSpec(move="rw", **work[4][1])]
    br = pkg.BatchRunner(specs)
    br.run(steps, graph=True)
    br.check()
    # tracking filters: the FP32 state against the single-problem FP32 filter
    # bit for bit (two independent FP32 runs drift apart by resampling flips,
    # so FP32 parity with the oracle is the lock-step test's), the stratified
    # FP64 filter against the oracle end to end
    kw = work[0][1]
    pf = pkg.ParticleFilter(kw["n"], kw["y"], seed=kw["seed"], problem_id=kw["problem_id"],
                            fp32_state=True)
    pf.run()
    hs = pf.history_host()
    cols = [L.SMC_H_ESS, L.SMC_H_FLAG, L.SMC_H_DLOGZ, L.SMC_H_LOGZ, L.SMC_H_L]
    assert np.array_equal(br.history_host(0)[:, cols], hs[:, cols])
    assert np.array_equal(br.state(0).cpu().numpy(), pf.state().cpu().numpy())
    pf.close()
    kw = work[1][1]
    cfg = orc.pf_cfg(kw["n"], kw["seed"], problem=kw["problem_id"], scheme="stratified")
    logz_o, hist_o, xf_o, _ = orc.pf_run(cfg, kw["y"])
    h = br.history_host(1)
    scale = max(1.0, np.abs(hist_o[:, 2]).sum())
    assert abs(br.log_z(1) - logz_o) <= 1e-12 * scale, (br.log_z(1), logz_o)
    assert np.array_equal(h[:steps + 1, L.SMC_H_FLAG], hist_o[:, 1])
    assert_close_l1(h[:steps + 1, L.SMC_H_ESS], hist_o[:, 0], hist_o[:, 0], 1e-11, "ess")
    # mixture samplers
    for i, (move, sweeps, scheme) in [(2, ("rw", 1, "stratified")), (3, ("mala", 2, "systematic")),
                                      (4, ("rw", 1, "systematic"))]:
        kw = work[i][1]
        sched = pkg.batch.gmm_schedule(kw["alphas"], None, move)
        cfg = orc.gmm_cfg(kw["n"], kw["seed"], kw["K"], problem=kw["problem_id"], move=move,
                          sweeps=sweeps, scheme=scheme)
        logz_o, hist_o, pop_o, _ = orc.gmm_run(cfg, kw["y"], sched[:, 0], sched[:, 1:])
        ts = assert_gmm_run_matches(br.history_host(i)[:steps + 1], hist_o, sched[:, 0], L,
                                    "problem %d" % i)
        assert ts == steps + 1, (i, ts)
        D = 3 * kw["K"] - 1
        st = br.state(i).cpu().numpy()[:D]
        assert_close_l1(st, pop_o, np.abs(pop_o) + 1.0, 1e-12, "problem %d population" % i)


def test_full_size_batched_workload_sampled(lib, orc):
    """The 128-filter / 32-sampler workload at its full sizes, a few steps:
    sampled problems against their single-problem runs, sampled particles'
    cached log-likelihoods against the oracle, weights and ESS bounds on
    every problem."""
    pkg, L = lib
    steps = 4
    work = synth.batched_workload(steps)
    specs = _specs(pkg, work)
    _say("full-size batch", len(specs), "problems")
    br = pkg.BatchRunner(specs)
    br.run(steps, graph=True)
    br.check()
    for i in range(len(work)):
        h = br.history_host(i)
        n = work[i][1]["n"]
        ess = h[:steps + 1, L.SMC_H_ESS]
        assert np.all(ess >= 1.0 - 1e-9) and np.all(ess <= n * (1 + 1e-12)), i
        assert np.all(np.isfinite(h[:steps + 1, L.SMC_H_LOGZ])), i
    pf_idx = [i for i, (k, _) in enumerate(work) if k == "pf"]
    gm_idx = [i for i, (k, _) in enumerate(work) if k == "gmm"]
    rng = np.random.default_rng(3)
    for i in list(rng.choice(pf_idx, 3, replace=False)):
        kw = work[i][1]
        pf = pkg.ParticleFilter(kw["n"], kw["y"][:steps + 1], seed=kw["seed"],
                                problem_id=kw["problem_id"])
        pf.run()
        assert pf.log_z() == br.log_z(i), i
    for i in list(rng.choice(gm_idx, 2, replace=False)):
        kw = work[i][1]
        s = pkg.GmmSampler(kw["n"], kw["y"], kw["K"], steps, seed=kw["seed"],
                           problem_id=kw["problem_id"], move="mala")
        s.run(kw["alphas"][:steps + 1])
        hs = s.history_host()
        scale = max(1.0, np.abs(hs[:, L.SMC_H_DLOGZ]).sum())
        assert abs(s.log_z() - br.log_z(i)) <= 1e-10 * scale, i
        # cached log-likelihood row of sampled particles against the oracle
        K = kw["K"]
        D = 3 * K - 1
        st = br.state(i).cpu().numpy()
        for j in rng.integers(0, kw["n"], 6):
            v = orc.gmm_loglik(st[:D, j], K, kw["y"])
            assert abs(st[D, j] - v) <= 1e-12 * (abs(v) + kw["y"].size), (i, j)
    # the oracle end to end on the smallest filter, all its observations
    small = min(pf_idx, key=lambda i: work[i][1]["n"])
    kw = work[small][1]
    logz_o, hist_o, _, _ = orc.pf_run(orc.pf_cfg(kw["n"], kw["seed"], problem=small),
                                      kw["y"][:steps + 1])
    assert abs(br.log_z(small) - logz_o) <= 1e-12 * max(1.0, np.abs(hist_o[:, 2]).sum())


def test_model_comparison_over_k(lib):
    # Section 5.2's purpose for the mixture example: the evidence of M_r for
    # several r from one batched run.  Data from two well-separated
    # components: one component explains them far worse (the gap is hundreds
    # of nats), and every batched evidence equals its single-problem run.
    pkg, L = lib
    y = synth.gmm_data(200, [-4.0, 4.0], 4.0, [0.5, 0.5], 77)
    T = 30
    alphas = synth.prior_tempering(T, 4.0)
    Ks = [1, 2, 3]
    specs = [pkg.GmmSpec(n=1 << 12, y=y, K=K, alphas=alphas, move="rw", seed=3,
                         problem_id=K) for K in Ks]
    br = pkg.BatchRunner(specs)
    br.run(T, graph=True)
    br.check()
    logz = [br.log_z(i) for i in range(len(Ks))]
    assert logz[1] - logz[0] > 100.0, logz
    for i, K in enumerate(Ks):
        s = pkg.GmmSampler(1 << 12, y, K, T, seed=3, problem_id=K, move="rw")
        s.run(alphas)
        scale = max(1.0, np.abs(s.history_host()[:, L.SMC_H_DLOGZ]).sum())
        assert abs(logz[i] - s.log_z()) <= 1e-10 * scale, (K, logz[i], s.log_z())
        s.close()
    br.close()
