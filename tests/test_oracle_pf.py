"""Pins of the oracle's tracking particle filter (Section 5.1, Algorithm
'pf'): observation densities against scipy, the whole filter against the
exact Kalman filter on the linear-Gaussian variant of the model."""
import math

import numpy as np
import pytest
from scipy import stats

import synth
from closed_forms import kalman_loglik


def test_student_t_logdensity(orc):
    cfg = orc.pf_cfg(1, 1)
    for pos, y in [(0.0, 0.0), (1.3, 1.1), (-2.0, 5.0), (0.5, 0.4999)]:
        ref = stats.t.logpdf(y, df=10, loc=pos, scale=0.1)
        assert orc.pf_obs_logdens(cfg, pos, y) == pytest.approx(ref, abs=1e-12)


def test_gaussian_logdensity(orc):
    cfg = orc.pf_cfg(1, 1, obs_nu=math.inf)
    for pos, y in [(0.0, 0.0), (1.3, 1.1), (-2.0, -1.0)]:
        ref = stats.norm.logpdf(y, loc=pos, scale=0.1)
        assert orc.pf_obs_logdens(cfg, pos, y) == pytest.approx(ref, abs=1e-12)


def test_paper_compatible_drops_constant(orc):
    a = orc.pf_cfg(1, 1)
    b = orc.pf_cfg(1, 1, paper_compatible=True)
    C = math.lgamma(5.5) - math.lgamma(5.0) - 0.5 * math.log(10 * math.pi) - math.log(0.1)
    assert 2 * C == pytest.approx(2.7173754816861884, abs=1e-14)
    for pos, y in [(0.1, 0.3), (2.0, -1.0)]:
        assert orc.pf_obs_logdens(a, pos, y) - orc.pf_obs_logdens(b, pos, y) == pytest.approx(C, abs=1e-13)
    # the paper's listing: -(nu+1)/2 log(1 + (10 r)^2 / nu)
    r = 0.3 - 0.1
    assert orc.pf_obs_logdens(b, 0.1, 0.3) == pytest.approx(-5.5 * math.log(1 + (10 * r) ** 2 / 10), abs=1e-14)


def test_init_moments(orc):
    cfg = orc.pf_cfg(200_000, 5, init_sd=(2.0, 2.0, 1.0, 1.0))
    x, lw = orc.pf_init(cfg, np.array([0.0, 0.0]))
    n = cfg.n
    for k, sd in enumerate([2.0, 2.0, 1.0, 1.0]):
        assert abs(x[k].mean()) < 5 * sd / math.sqrt(n)
        assert abs(x[k].var() / sd ** 2 - 1) < 5 * math.sqrt(2 / n)
    assert abs(np.corrcoef(x)[0, 1]) < 5 / math.sqrt(n)


def test_move_one_step_kalman_moments(orc):
    # from a fixed point the move gives N(A x, Q) (positions use the old velocity)
    n = 200_000
    cfg = orc.pf_cfg(n, 9)
    x0 = np.tile(np.array([[1.0], [-2.0], [3.0], [0.5]]), (1, n))
    x1, _ = orc.pf_move(cfg, 4, np.array([0.0, 0.0]), x0, np.zeros(n), True)
    mean = np.array([1.0 + 0.1 * 3.0, -2.0 + 0.1 * 0.5, 3.0, 0.5])
    sd = np.array([0.02, 0.02, 0.5, 0.5])
    assert np.all(np.abs(x1.mean(axis=1) - mean) < 5 * sd / math.sqrt(n))
    assert np.all(np.abs(x1.std(axis=1) / sd - 1) < 0.02)


def test_move_one_step_moments_fp32(orc):
    # the FP32-state branch: float normals, float transition from a fixed
    # point.  Mean A x with the old velocity (a dropped dt moves the position
    # mean by 0.9 x_vel), position sd 0.02 alone (the new velocity in the
    # position update would make it sqrt(0.02^2 + (0.1 * 0.5)^2) = 0.054),
    # independent coordinates, float-representable results.
    n = 200_000
    cfg = orc.pf_cfg(n, 9, fp32_state=True)
    x0 = np.tile(np.array([[1.0], [-2.0], [3.0], [0.5]]), (1, n))
    y = np.array([1.25, -1.9])
    x1, lw1 = orc.pf_move(cfg, 4, y, x0, np.zeros(n), True)
    assert np.array_equal(x1.astype(np.float32).astype(np.float64), x1)
    mean = np.array([1.0 + 0.1 * 3.0, -2.0 + 0.1 * 0.5, 3.0, 0.5])
    sd = np.array([0.02, 0.02, 0.5, 0.5])
    # float rounding of the mean itself: a few ulp of |x| ~ 1e-7, far inside
    assert np.all(np.abs(x1.mean(axis=1) - mean) < 5 * sd / math.sqrt(n) + 1e-6)
    assert np.all(np.abs(x1.std(axis=1) / sd - 1) < 0.02)
    c = np.corrcoef(x1)
    assert np.all(np.abs(c[np.triu_indices(4, 1)]) < 5 / math.sqrt(n))
    # the increment is the FP64 observation density at the new float position
    for i in range(0, n, 20_000):
        ref = (stats.t.logpdf(y[0], df=10, loc=x1[0, i], scale=0.1) +
               stats.t.logpdf(y[1], df=10, loc=x1[1, i], scale=0.1))
        assert lw1[i] == pytest.approx(ref, abs=1e-11)
    # the float noise does not reuse the FP64 stream's values
    x64, _ = orc.pf_move(orc.pf_cfg(n, 9), 4, y, x0, np.zeros(n), True)
    assert not np.allclose(x1[2], x64[2], rtol=0, atol=1e-3)


def test_init_moments_fp32(orc):
    cfg = orc.pf_cfg(200_000, 5, init_sd=(2.0, 2.0, 1.0, 1.0), fp32_state=True)
    y0 = np.array([0.3, -0.2])
    x, lw = orc.pf_init(cfg, y0)
    n = cfg.n
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    for k, sd in enumerate([2.0, 2.0, 1.0, 1.0]):
        assert abs(x[k].mean()) < 5 * sd / math.sqrt(n)
        assert abs(x[k].var() / sd ** 2 - 1) < 5 * math.sqrt(2 / n)
    c = np.corrcoef(x)
    assert np.all(np.abs(c[np.triu_indices(4, 1)]) < 5 / math.sqrt(n))
    for i in range(0, n, 40_000):
        ref = (stats.t.logpdf(y0[0], df=10, loc=x[0, i], scale=0.1) +
               stats.t.logpdf(y0[1], df=10, loc=x[1, i], scale=0.1))
        assert lw[i] == pytest.approx(ref, abs=1e-11)


def test_lw_reset_and_accumulate(orc):
    rng = np.random.default_rng(0)
    n = 100
    cfg = orc.pf_cfg(n, 3)
    x = rng.normal(size=(4, n))
    lw = rng.normal(size=n)
    y = np.array([0.2, -0.1])
    x1, a = orc.pf_move(cfg, 2, y, x, lw, False)
    _, b = orc.pf_move(cfg, 2, y, x, lw, True)
    assert np.allclose(a - b, lw, rtol=0, atol=1e-12)
    inc = np.array([orc.pf_obs_logdens(cfg, x1[0, i], y[0]) + orc.pf_obs_logdens(cfg, x1[1, i], y[1])
                    for i in range(n)])
    assert np.allclose(b, inc, rtol=0, atol=1e-12)


def _kf_case(T, data_seed):
    model = synth.CVModel(obs_nu=math.inf)
    _, y = synth.pf_trajectory(T, data_seed, model)
    ll, means = kalman_loglik(y, model.dt, model.sd_pos, model.sd_vel, model.obs_scale, model.init_sd)
    return y, ll, means


@pytest.mark.parametrize("scheme,fp32", [("systematic", False), ("multinomial", False),
                                         ("systematic", True), ("multinomial", True)])
def test_filter_log_evidence_matches_kalman(orc, scheme, fp32):
    # PF log Z is unbiased for Z; over several seeds it sits within a few
    # standard errors of the exact Kalman-filter log p(y_0..T-1).  The
    # FP32-state variant (float state, draws and transition; FP64 weights)
    # must reach the same evidence: its rounding (~1e-7 of the state) is far
    # below the Monte Carlo error, while a dropped term of its transition
    # moves log Z by many standard errors.
    T = 40
    y, ll_kf, means_kf = _kf_case(T, 4242)
    vals = []
    est_means = []
    for seed in range(1, 9):
        cfg = orc.pf_cfg(1 << 14, seed, obs_nu=math.inf, scheme=scheme, fp32_state=fp32)
        logz, hist, _, _ = orc.pf_run(cfg, y)
        vals.append(logz)
        est_means.append(hist[:, 5:9])
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(vals.size)
    assert abs(vals.mean() - ll_kf) < 4 * se + 0.02
    est_means = np.array(est_means)
    em = est_means.mean(axis=0)
    se_m = est_means.std(axis=0, ddof=1) / math.sqrt(est_means.shape[0])
    # filtered means within Monte Carlo error of the exact filtered means
    assert np.all(np.abs(em - means_kf) < 6 * se_m + 1e-3)


def test_filter_history_consistency(orc):
    _, y = synth.pf_trajectory(30, 7)
    cfg = orc.pf_cfg(2000, 1)
    logz, hist, xf, lwf = orc.pf_run(cfg, y)
    assert logz == pytest.approx(hist[:, 2].sum(), abs=1e-10)
    assert logz == pytest.approx(hist[-1, 3], abs=0)
    assert np.all((hist[:, 0] >= 1 - 1e-9) & (hist[:, 0] <= 2000 * (1 + 1e-12)))
    assert np.array_equal(hist[:, 1] == 1, hist[:, 0] < 1000)
    # always / never resample
    c1 = orc.pf_cfg(500, 2, threshold=1.0)
    _, h1, _, lw1 = orc.pf_run(c1, y)
    assert np.all(h1[:, 1] == 1) and np.all(lw1 == 0)
    c0 = orc.pf_cfg(500, 2, threshold=0.0)
    z0, h0, _, lw0 = orc.pf_run(c0, y)
    assert np.all(h0[:, 1] == 0)
    # without resampling, log Z = log mean exp(sum of increments)
    assert z0 == pytest.approx(orc.lse(lw0) - math.log(500), abs=1e-9)


def test_fp32_state_close_to_fp64(orc):
    _, y = synth.pf_trajectory(5, 3)
    n = 1000
    c64 = orc.pf_cfg(n, 4)
    c32 = orc.pf_cfg(n, 4, fp32_state=True)
    x64, lw64 = orc.pf_init(c64, y[0])
    x32, lw32 = orc.pf_init(c32, y[0])
    # state values are float-representable
    assert np.array_equal(x32.astype(np.float32).astype(np.float64), x32)
    # the FP32 variant draws its normals differently; compare distributions only
    assert abs(x32.std() - x64.std()) < 0.1


@pytest.mark.parametrize("scheme", ["systematic", "multinomial", "stratified"])
def test_results_do_not_depend_on_threads(orc, scheme):
    # per-particle loops may run on several threads, every sum stays
    # sequential in index order: one thread and many give the same bits
    _, y = synth.pf_trajectory(6, 3)
    runs = []
    n0 = orc.max_threads()
    for th in (1, 4):
        orc.set_threads(th)
        runs.append(orc.pf_run(orc.pf_cfg(20011, 2, scheme=scheme), y))
    orc.set_threads(n0)
    assert runs[0][0] == runs[1][0]
    for a, b in zip(runs[0][1:], runs[1][1:]):
        assert np.array_equal(a, b)
