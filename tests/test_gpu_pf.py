"""GPU parity of the tracking particle filter path (Section 5.1) against the
oracle, through the C ABI: Philox words, prior draws, the fused move +
weight sweep, normalisation, resampling (systematic / multinomial /
stratified), monitors; lock-step over whole runs, end-to-end at N = 1000,
determinism and edge cases."""
import math
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import assert_ancestors, assert_close_l1, decision_matches

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_5583_amd as pkg
    from paper_1306_5583_amd import _lib
    _lib.load()
    return pkg, _lib


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_philox_words_bit_exact(lib, orc):
    pkg, L = lib
    n = 5000
    for (seed, t, tag, call, p) in [(1, 0, 1, 0, 0), (0xDEADBEEFCAFEF00D, 123, 7, 1, 5),
                                    (42, 7, 2, 1, 0), (2 ** 64 - 1, 2 ** 20, 6, 65535, 2 ** 32 - 1)]:
        out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
        L.smc_draw_words(seed, t, tag, call, p, n, out.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
        got = out.cpu().numpy().view(np.uint32).reshape(n, 4)
        for i in list(range(0, n, 97)) + [n - 1]:
            ref = orc.draw_words(seed, i, t, tag, call, p)
            assert list(got[i]) == list(ref), (seed, t, tag, call, p, i)


def _gathered(state, anc, resampled):
    return state[:, anc] if resampled else state


def _lockstep(lib, orc, n, T, seed, scheme, fp32=False, obs_nu=10.0, threshold=0.5, data_seed=7,
              fused_monitor=False):
    """Runs the GPU filter step by step; at every step the oracle recomputes
    the step from the GPU's input state and the outputs are compared.  With
    fused_monitor the monitor of step t rides on the move of step t + 1 and
    is completed by its normalisation (the benchmark's launch sequence);
    otherwise each step calls the standalone monitor."""
    pkg, L = lib
    _say("lockstep n=%d T=%d seed=%d scheme=%s fp32=%s nu=%s thr=%s fused_monitor=%s" %
         (n, T, seed, scheme, fp32, obs_nu, threshold, fused_monitor))
    model = synth.CVModel(obs_nu=obs_nu)
    _, y = synth.pf_trajectory(T, data_seed, model)
    pf = pkg.ParticleFilter(n, y, seed=seed, scheme=scheme, fp32_state=fp32, obs_nu=obs_nu,
                            threshold=threshold)
    ocfg = orc.pf_cfg(n, seed, scheme=scheme, fp32_state=fp32, obs_nu=obs_nu, threshold=threshold)
    rtol = 1e-5 if fp32 else 1e-12
    ctx = pf.ctx
    L.smc_init(ctx)
    torch.cuda.synchronize()
    x_g = pf.state().double().cpu().numpy()
    lw_g = pf.log_weight.cpu().numpy()
    x_o, lw_o = orc.pf_init(ocfg, y[0])
    assert_close_l1(x_g, x_o, np.abs(x_o), rtol, "init state")
    assert_close_l1(lw_g, lw_o, np.abs(lw_o), rtol, "init lw")
    logz_scale = 0.0
    flips = 0
    resampled = False
    est_prev = None
    for t in range(T):
        if t > 0:
            x_in = _gathered(x_g, anc_g, resampled)
            lw_in = lw_g
            pf._margs.obs_index = t
            pf._margs.monitor_step = t - 1 if fused_monitor else -1
            L.smc_move(ctx, t, pf._margs)
            torch.cuda.synchronize()
            x_g = pf.state().double().cpu().numpy()
            lw_g = pf.log_weight.cpu().numpy()
            x_o, lw_o = orc.pf_move(ocfg, t, y[t], x_in, lw_in, resampled)
            sx = np.abs(x_in) + np.abs(x_o) + 0.1 * np.abs(x_in[[2, 3, 2, 3]])
            assert_close_l1(x_g, x_o, sx, rtol, "state t=%d" % t)
            inc = lw_o - (0.0 if resampled else lw_in)
            sl = np.abs(inc) + (0.0 if resampled else np.abs(lw_in)) + 10.0
            assert_close_l1(lw_g, lw_o, sl, 1e-12 if not fp32 else rtol, "lw t=%d" % t)
        # normalisation on the GPU's weights
        L.smc_ess(ctx, t)
        sc = pf.scalars_host()
        if fused_monitor and t > 0:
            # the monitor of step t - 1, completed alongside this normalisation
            hist = pf.history.cpu().numpy()
            assert_close_l1(hist[t - 1, L.SMC_H_MON:L.SMC_H_MON + 4], est_prev[0], est_prev[1],
                            rtol, "fused monitor t=%d" % (t - 1))
        Lo, L2o, esso = orc.normalise(lw_g)
        assert abs(sc[L.SMC_S_L] - Lo) <= 1e-12 * max(1.0, abs(Lo)), (t, sc[L.SMC_S_L], Lo)
        assert abs(sc[L.SMC_S_ESS] - esso) <= 1e-12 * esso, (t, sc[L.SMC_S_ESS], esso)
        logz_scale += abs(sc[L.SMC_S_DLOGZ])
        flag_o = orc.resample_flag(esso, n, threshold)
        assert decision_matches(sc[L.SMC_S_FLAG], flag_o, esso, threshold * n), t
        L.smc_resample(ctx, t)
        torch.cuda.synchronize()
        sc = pf.scalars_host()
        resampled = sc[L.SMC_S_RESAMPLED] != 0.0
        assert resampled == bool(sc[L.SMC_S_FLAG])
        anc_g = pf.ancestors.cpu().numpy().astype(np.int64)
        if resampled:
            anc_o, S_o, u_o = orc.resample(scheme, seed, t, lw_g)
            if scheme == "systematic":
                w = orc.draw_words(seed, 0, t, orc.TAG_RESAMPLE, 0)
                assert sc[L.SMC_S_U] == orc.u53(int(w[0]), int(w[1]))
            flips += assert_ancestors(anc_g, anc_o, S_o, u_o, what="anc t=%d" % t)
        # monitor after resampling
        xm = _gathered(x_g, anc_g, resampled)
        lwm = np.zeros(n) if resampled else lw_g
        est_o = orc.weighted_mean(xm, lwm)
        mon_scale = np.abs(xm).max(axis=1) * 4
        if fused_monitor and t < T - 1:
            est_prev = (est_o, mon_scale)
            continue
        out = torch.zeros(4, dtype=torch.float64, device="cuda")
        L.smc_monitor(ctx, t, out.data_ptr())
        torch.cuda.synchronize()
        est_g = out.cpu().numpy()
        assert_close_l1(est_g, est_o, mon_scale, rtol, "monitor t=%d" % t)
        hist = pf.history.cpu().numpy()
        assert np.array_equal(hist[t, L.SMC_H_MON:L.SMC_H_MON + 4], est_g)
    pf.check()
    _say("  ancestor boundary flips: %d" % flips)
    return pf


@pytest.mark.parametrize("n,scheme", [(1000, "systematic"), (5000, "systematic"),
                                      (5000, "multinomial"), (3077, "stratified"),
                                      (70001, "systematic"), (70001, "multinomial")])
def test_lockstep_fp64(lib, orc, n, scheme):
    _lockstep(lib, orc, n, 25, 11, scheme)


@pytest.mark.parametrize("n,scheme", [(4099, "systematic"), (4099, "multinomial")])
def test_lockstep_fp32_state(lib, orc, n, scheme):
    _lockstep(lib, orc, n, 15, 5, scheme, fp32=True)


def test_lockstep_gaussian_obs(lib, orc):
    _lockstep(lib, orc, 2048, 15, 3, "systematic", obs_nu=math.inf)


@pytest.mark.parametrize("threshold", [0.0, 1.0, 0.999])
def test_lockstep_thresholds(lib, orc, threshold):
    _lockstep(lib, orc, 1500, 8, 4, "systematic", threshold=threshold)


@pytest.mark.parametrize("n", [1, 2, 63, 1024, 1025])
def test_small_and_tile_edges(lib, orc, n):
    _lockstep(lib, orc, n, 6, 9, "systematic", threshold=1.0)


def test_full_size_lockstep_steps(lib, orc):
    # the benchmark's workload: N = 2^22, its launch sequence (monitor fused
    # into the next move), a few full steps in lock-step
    _lockstep(lib, orc, 1 << 22, 4, 2, "systematic", fused_monitor=True)


def test_full_size_multinomial(lib, orc):
    _lockstep(lib, orc, 1 << 22, 3, 3, "multinomial", threshold=1.0, fused_monitor=True)


@pytest.mark.parametrize("scheme", ["systematic", "multinomial"])
def test_full_size_fp32_state(lib, orc, scheme):
    # the FP32-state variant of the same workload (threshold 1: every step
    # resamples, so the gathered FP32 path runs on each)
    _lockstep(lib, orc, 1 << 22, 3, 6, scheme, fp32=True, threshold=1.0, fused_monitor=True)


def test_lockstep_fused_monitor_small(lib, orc):
    # the benchmark's launch sequence over a ragged population, many steps
    _lockstep(lib, orc, 70001, 20, 12, "systematic", fused_monitor=True)


def test_end_to_end_c0(lib, orc):
    # the N = 1000, T = 100 filter run independently on both sides
    pkg, L = lib
    _, y = synth.pf_trajectory(100, synth.DATA_SEED[0])
    pf = pkg.ParticleFilter(1000, y, seed=1)
    logz_g = pf.run()
    hist_g = pf.history_host()
    ocfg = orc.pf_cfg(1000, 1)
    logz_o, hist_o, xf_o, lwf_o = orc.pf_run(ocfg, y)
    assert abs(logz_g - logz_o) <= 1e-12 * max(1.0, np.abs(hist_o[:, 2]).sum())
    assert np.array_equal(hist_g[:, L.SMC_H_FLAG], hist_o[:, 1])
    assert_close_l1(hist_g[:, L.SMC_H_ESS], hist_o[:, 0], hist_o[:, 0], 1e-11, "ess")
    assert_close_l1(hist_g[:, L.SMC_H_MON:L.SMC_H_MON + 4], hist_o[:, 5:9], 20.0, 1e-11, "means")
    pf.check()


@pytest.mark.parametrize("n", [1, 63, 1000, 1024])
@pytest.mark.parametrize("scheme,fp32", [("systematic", False), ("stratified", False),
                                         ("systematic", True)])
def test_one_launch_step_matches_three_calls(lib, n, scheme, fp32):
    # smc_step of a one-tile filter (one launch: move + weight, normalisation
    # with the carried monitor, resampling) against smc_move, smc_ess and
    # smc_resample, bit for bit over a whole run; thresholds 0.5 and 1 (a
    # resample every step)
    pkg, L = lib
    _, y = synth.pf_trajectory(30, 5)
    for thr in (0.5, 1.0):
        _say("one-launch step", n, scheme, fp32, thr)
        a = pkg.ParticleFilter(n, y, seed=3, scheme=scheme, fp32_state=fp32, threshold=thr)
        b = pkg.ParticleFilter(n, y, seed=3, scheme=scheme, fp32_state=fp32, threshold=thr)
        a.run()
        b.init()
        mon = 0
        for t in range(1, b.T):
            m = b._margs
            m.obs_index, m.monitor_step = t, mon
            L.smc_move(b.ctx, t, m)
            L.smc_ess(b.ctx, t)
            L.smc_resample(b.ctx, t)
            mon = t
        b._mon_pending = mon
        b.finish()
        ha, hb = a.history_host(), b.history_host()
        assert np.array_equal(ha, hb)
        for u, v in [(a.state(), b.state()), (a.log_weight, b.log_weight),
                     (a.ancestors, b.ancestors)]:
            assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())
        assert a.log_z() == b.log_z()
        if thr == 1.0:
            assert np.all(ha[1:, L.SMC_H_FLAG] == 1.0)
        a.check()
        b.check()


@pytest.mark.parametrize("scheme,n", [("systematic", 1000), ("multinomial", 5003)])
def test_captured_run_replays_match_eager(lib, scheme, n):
    # the whole run captured as one graph and replayed three times, with the
    # filter run eagerly and the host synchronised between replays: every
    # replay reproduces the eager run bit for bit
    pkg, L = lib
    _, y = synth.pf_trajectory(60, synth.DATA_SEED[0])
    pf = pkg.ParticleFilter(n, y, seed=1, scheme=scheme)
    logz_e = pf.run()
    ref = [pf.history_host().copy(), pf.state().cpu().numpy().copy(),
           pf.log_weight.cpu().numpy().copy(), pf.ancestors.cpu().numpy().copy()]
    g = pf.capture_run()
    for r in range(3):
        if r == 1:
            assert pf.run() == logz_e
        _say("replay", r, scheme, n)
        g.replay()
        torch.cuda.synchronize()
        assert pf.log_z() == logz_e
        got = [pf.history_host(), pf.state().cpu().numpy(), pf.log_weight.cpu().numpy(),
               pf.ancestors.cpu().numpy()]
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
    pf.check()


def test_deterministic(lib):
    pkg, L = lib
    _, y = synth.pf_trajectory(40, 3)
    runs = []
    for _ in range(2):
        pf = pkg.ParticleFilter(100_000, y, seed=8, scheme="multinomial")
        pf.run()
        torch.cuda.synchronize()
        runs.append((pf.history_host().copy(), pf.state().cpu().numpy().copy(),
                     pf.log_weight.cpu().numpy().copy(), pf.ancestors.cpu().numpy().copy()))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


def test_unfused_reweight_matches_fused(lib):
    pkg, L = lib
    _, y = synth.pf_trajectory(10, 3)
    a = pkg.ParticleFilter(3000, y, seed=2)
    b = pkg.ParticleFilter(3000, y, seed=2)
    a.init()
    b.init()
    L.smc_monitor(b.ctx, 0)
    for t in range(1, 10):
        a.step(t)
        m = L.smc_move_args()
        m.obs_index, m.fuse_reweight = t, 0
        L.smc_move(b.ctx, t, m)
        r = L.smc_reweight_args()
        r.obs_index = t
        L.smc_reweight(b.ctx, t, r)
        L.smc_ess(b.ctx, t)
        L.smc_resample(b.ctx, t)
        L.smc_monitor(b.ctx, t)
    a.finish()
    torch.cuda.synchronize()
    ha, hb = a.history_host(), b.history_host()
    assert np.array_equal(ha[:, :L.SMC_H_MON], hb[:, :L.SMC_H_MON])
    # a's monitors come from the fused sweep, b's from the standalone kernels
    assert_close_l1(ha[:, L.SMC_H_MON:L.SMC_H_MON + 4], hb[:, L.SMC_H_MON:L.SMC_H_MON + 4], 20.0,
                    1e-14, "fused monitor")
    assert torch.equal(a.state(), b.state()) and torch.equal(a.log_weight, b.log_weight)


@pytest.mark.parametrize("fp32,threshold", [(False, 0.5), (True, 0.5), (False, 0.0)])
def test_fused_monitor_matches_standalone(lib, fp32, threshold):
    pkg, L = lib
    _, y = synth.pf_trajectory(30, 5)
    a = pkg.ParticleFilter(9000, y, seed=4, fp32_state=fp32, threshold=threshold)
    b = pkg.ParticleFilter(9000, y, seed=4, fp32_state=fp32, threshold=threshold)
    a.run()
    b.init()
    L.smc_monitor(b.ctx, 0)
    for t in range(1, 30):
        m = L.smc_move_args()
        m.obs_index, m.fuse_reweight = t, 1
        L.smc_move(b.ctx, t, m)
        L.smc_ess(b.ctx, t)
        L.smc_resample(b.ctx, t)
        L.smc_monitor(b.ctx, t)
    ha, hb = a.history_host(), b.history_host()
    assert np.array_equal(ha[:, :L.SMC_H_MON], hb[:, :L.SMC_H_MON])
    assert_close_l1(ha[:, L.SMC_H_MON:L.SMC_H_MON + 4], hb[:, L.SMC_H_MON:L.SMC_H_MON + 4], 20.0,
                    1e-14, "fused monitor")


def test_gather_materialises_state(lib, orc):
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    pf = pkg.ParticleFilter(2500, y, seed=2, threshold=1.0)
    pf.init()
    torch.cuda.synchronize()
    before = pf.state().cpu().numpy().copy()
    anc = pf.ancestors.cpu().numpy().astype(np.int64)
    L.smc_gather(pf.ctx)
    torch.cuda.synchronize()
    assert np.array_equal(pf.state().cpu().numpy(), before[:, anc])


@pytest.mark.parametrize("n,far", [(2500, False), (70001, False), (70001, True),
                                   (1 << 22, False)])
def test_copy_from_layout_matches_oracle(lib, orc, n, far):
    # the in-place parent layout of Section 4.1 from the sorted ancestors,
    # bit-exact against the oracle's derivation; `far` puts the first
    # observation far from every particle so that a handful of parents take
    # almost all slots (long runs of duplicates, mostly empty particles)
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    if far:
        y = y.copy()
        y[0] = (6.0, 6.0)
    pf = pkg.ParticleFilter(n, y, seed=4, threshold=1.0)
    pf.init()
    cf = pf.copy_from().cpu().numpy()
    anc = pf.ancestors.cpu().numpy()
    assert pf.scalars_host()[L.SMC_S_RESAMPLED] == 1.0
    assert np.array_equal(cf, orc.copy_from(anc))
    if far:
        assert np.unique(anc).size < n // 10
    pf.close()


def test_copy_from_identity_without_resample(lib):
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    pf = pkg.ParticleFilter(3000, y, seed=4, threshold=0.0)
    pf.init()
    assert pf.scalars_host()[L.SMC_S_RESAMPLED] == 0.0
    assert np.array_equal(pf.copy_from().cpu().numpy(), np.arange(3000, dtype=np.int32))
    pf.close()


def test_force_resample_and_error_word(lib):
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    pf = pkg.ParticleFilter(3000, y, seed=2, threshold=0.0)
    pf.init()
    sc = pf.scalars_host()
    assert sc[L.SMC_S_RESAMPLED] == 0.0
    # force a resample although the rule says never
    m = L.smc_move_args()
    m.obs_index, m.fuse_reweight = 1, 1
    L.smc_move(pf.ctx, 1, m)
    L.smc_ess(pf.ctx, 1)
    L.smc_resample(pf.ctx, 1, force=True)
    sc = pf.scalars_host()
    assert sc[L.SMC_S_RESAMPLED] == 1.0 and sc[L.SMC_S_L] == pytest.approx(math.log(3000))
    pf.check()
    # all log-weights -inf: the normalisation raises the device error word
    L.smc_move(pf.ctx, 2, m)
    pf.log_weight.fill_(-math.inf)
    r = L.smc_reweight_args()
    r.obs_index = 2
    L.smc_reweight(pf.ctx, 2, r)
    L.smc_ess(pf.ctx, 2)
    L.smc_resample(pf.ctx, 2, force=True)
    with pytest.raises(L.SmcError) as e:
        pf.check()
    assert e.value.status == L.SMC_ERR_NUMERIC


def test_out_of_order_calls_rejected(lib):
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    pf = pkg.ParticleFilter(100, y, seed=2)
    with pytest.raises(L.SmcError) as e:
        L.smc_resample(pf.ctx, 0)
    assert e.value.status == L.SMC_ERR_BAD_STATE
    L.smc_init(pf.ctx)
    m = L.smc_move_args()
    m.obs_index = 99
    with pytest.raises(L.SmcError) as e:
        L.smc_move(pf.ctx, 1, m)
    assert e.value.status == L.SMC_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [100, 5000])
def test_step_rejects_what_the_three_calls_reject(lib, n):
    # smc_step's checks, in its one-launch form (n = 100) and as the three
    # calls (n = 5000): before init, a bad observation row, a negative step
    pkg, L = lib
    _, y = synth.pf_trajectory(5, 3)
    pf = pkg.ParticleFilter(n, y, seed=2)
    m = L.smc_move_args()
    m.obs_index, m.fuse_reweight = 1, 1
    with pytest.raises(L.SmcError) as e:
        L.smc_step(pf.ctx, 1, m)
    assert e.value.status == L.SMC_ERR_BAD_STATE
    pf.init()
    m.fuse_reweight = 0  # the step's normalisation needs the move's weights
    with pytest.raises(L.SmcError) as e:
        L.smc_step(pf.ctx, 1, m)
    assert e.value.status == L.SMC_ERR_INVALID_ARG
    m.fuse_reweight = 1
    m.obs_index = 99
    with pytest.raises(L.SmcError) as e:
        L.smc_step(pf.ctx, 1, m)
    assert e.value.status == L.SMC_ERR_INVALID_ARG
    m.obs_index = 1
    with pytest.raises(L.SmcError) as e:
        L.smc_step(pf.ctx, -1, m)
    assert e.value.status == L.SMC_ERR_INVALID_ARG
    # after the rejected calls the filter still steps and stays consistent
    m.monitor_step = 0
    L.smc_step(pf.ctx, 1, m)
    L.smc_monitor(pf.ctx, 1)
    pf.check()


def test_move_kernel_profile_events(lib):
    # dispatch-carried timing of the move kernel: one duration per timed launch
    pkg, L = lib
    _, y = synth.pf_trajectory(12, 3)
    pf = pkg.ParticleFilter(1 << 16, y, seed=2)
    pf.init()
    L.smc_profile_start(pf.ctx, 5)
    for t in range(1, 12):
        pf.step(t)
    pf.finish()
    ms = L.smc_profile_read(pf.ctx, 16)
    assert len(ms) == 5 and all(0.0 < v < 50.0 for v in ms)
    L.smc_profile_start(pf.ctx, 0)
    assert L.smc_profile_read(pf.ctx, 4) == []
    pf.check()
