"""Pins of the oracle's Gaussian-mixture sampler (Section 5.2): the mixture
likelihood against a brute-force allocation sum, its gradient against
finite differences, the prior (with both change-of-variable Jacobians)
against scipy densities and a numerical Jacobian, the sampler's invariance
of the prior at tempering exponent 0, and the evidence of a one-component
model against quadrature."""
import math

import numpy as np
import pytest
from scipy import special, stats

import synth
from closed_forms import gmm_k1_log_evidence, gmm_loglik_bruteforce


def _phi(mu, lam, w):
    mu, lam, w = map(np.asarray, (mu, lam, w))
    return np.concatenate([mu, np.log(lam), np.log(w[:-1]) - np.log(w[-1])])


@pytest.mark.parametrize("K,n", [(1, 4), (2, 5), (3, 6), (2, 1)])
def test_loglik_bruteforce(orc, K, n):
    rng = np.random.default_rng(K * 10 + n)
    for _ in range(3):
        y = rng.normal(0, 2, n)
        mu = rng.normal(0, 2, K)
        lam = rng.gamma(2.0, 1.0, K)
        w = rng.dirichlet(np.ones(K))
        ref = gmm_loglik_bruteforce(y, mu, lam, w)
        got = orc.gmm_loglik(_phi(mu, lam, w), K, y)
        assert got == pytest.approx(ref, abs=1e-11 * max(1, abs(ref)))


def test_loglik_far_components_stable(orc):
    # points far from every component: the naive sum of exps underflows, the
    # per-point log-sum-exp does not
    y = np.array([200.0, -150.0])
    mu, lam, w = np.array([0.0, 1.0]), np.array([50.0, 40.0]), np.array([0.3, 0.7])
    got = orc.gmm_loglik(_phi(mu, lam, w), 2, y)
    ref = sum(special.logsumexp([math.log(w[j]) + stats.norm.logpdf(yk, mu[j], 1 / math.sqrt(lam[j]))
                                 for j in range(2)]) for yk in y)
    assert np.isfinite(got) and got == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("K", [1, 2, 4, 6])
def test_loglik_gradient_finite_differences(orc, K):
    rng = np.random.default_rng(K)
    y = synth.gmm_data(200, np.linspace(-3, 3, max(K, 1)), 1.5, np.ones(max(K, 1)), K)
    phi = np.concatenate([rng.normal(0, 2, K), rng.normal(0, 0.5, K), rng.normal(0, 0.5, K - 1)])
    v, g = orc.gmm_loglik(phi, K, y, grad=True)
    assert v == orc.gmm_loglik(phi, K, y)
    h = 1e-6
    for q in range(3 * K - 1):
        e = np.zeros_like(phi)
        e[q] = h
        fd = (orc.gmm_loglik(phi + e, K, y) - orc.gmm_loglik(phi - e, K, y)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * abs(g[q]) + 1e-4


def _constrained_logdens(phi, K, cfg):
    mu, eta, z = phi[:K], phi[K:2 * K], phi[2 * K:]
    lam = np.exp(eta)
    w = np.exp(np.append(z, 0.0) - special.logsumexp(np.append(z, 0.0)))
    out = stats.norm.logpdf(mu, cfg.mu_mean, cfg.mu_sd).sum()
    out += stats.gamma.logpdf(lam, a=cfg.gamma_shape, scale=1 / cfg.gamma_rate).sum()
    if K > 1:
        out += stats.dirichlet.logpdf(w, np.full(K, cfg.dir_rho))
    return out


def _map(phi, K):
    # phi -> (mu, lambda, omega_1..omega_{K-1}), the coordinates the prior is stated in
    mu, eta, z = phi[:K], phi[K:2 * K], phi[2 * K:]
    w = np.exp(np.append(z, 0.0) - special.logsumexp(np.append(z, 0.0)))
    return np.concatenate([mu, np.exp(eta), w[:-1]])


def _log_abs_jac(phi, K):
    D = phi.size
    J = np.zeros((D, D))
    h = 1e-6
    for q in range(D):
        e = np.zeros(D)
        e[q] = h
        J[:, q] = (_map(phi + e, K) - _map(phi - e, K)) / (2 * h)
    return np.linalg.slogdet(J)[1]


@pytest.mark.parametrize("K", [1, 2, 3, 5])
@pytest.mark.parametrize("hyper", [(0.0, 10.0, 1.0, 1.0, 1.0), (1.0, 3.0, 2.5, 0.5, 2.0)])
def test_logprior_matches_density_and_jacobian(orc, K, hyper):
    m, s, a, b, rho = hyper
    cfg = orc.gmm_cfg(1, 1, K, mu_mean=m, mu_sd=s, gamma_shape=a, gamma_rate=b, dir_rho=rho)
    rng = np.random.default_rng(K)
    pts = [np.concatenate([rng.normal(0, 2, K), rng.normal(0, 0.7, K), rng.normal(0, 0.7, K - 1)])
           for _ in range(4)]
    ref = [_constrained_logdens(p, K, cfg) + _log_abs_jac(p, K) for p in pts]
    got = [orc.gmm_logprior(cfg, p) for p in pts]
    for q in range(1, len(pts)):   # the prior is defined up to a constant
        assert got[q] - got[0] == pytest.approx(ref[q] - ref[0], abs=1e-6)


@pytest.mark.parametrize("K", [1, 3, 5])
def test_logprior_gradient_finite_differences(orc, K):
    cfg = orc.gmm_cfg(1, 1, K, mu_mean=0.5, mu_sd=4.0, gamma_shape=2.0, gamma_rate=0.7, dir_rho=1.5)
    rng = np.random.default_rng(7)
    phi = np.concatenate([rng.normal(0, 2, K), rng.normal(0, 0.5, K), rng.normal(0, 0.5, K - 1)])
    _, g = orc.gmm_logprior(cfg, phi, grad=True)
    h = 1e-6
    for q in range(3 * K - 1):
        e = np.zeros_like(phi)
        e[q] = h
        fd = (orc.gmm_logprior(cfg, phi + e) - orc.gmm_logprior(cfg, phi - e)) / (2 * h)
        assert fd == pytest.approx(g[q], abs=1e-6)


def _prior_moment_check(pop, K, n):
    mu, eta, z = pop[:K], pop[K:2 * K], pop[2 * K:]
    lam = np.exp(eta)
    zz = np.vstack([z, np.zeros((1, n))])
    w = np.exp(zz - special.logsumexp(zz, axis=0))
    se = lambda v: math.sqrt(v / n)
    assert np.all(np.abs(mu.mean(axis=1)) < 5 * se(100.0))
    assert np.all(np.abs(mu.var(axis=1) - 100.0) < 5 * 100 * math.sqrt(2 / n))
    assert np.all(np.abs(lam.mean(axis=1) - 1.0) < 5 * se(1.0))
    assert np.all(np.abs(lam.var(axis=1) - 1.0) < 5 * math.sqrt(8.0 / n))  # var of var, Exp(1)
    vw = (K - 1) / (K * K * (K + 1))
    assert np.all(np.abs(w.mean(axis=1) - 1.0 / K) < 5 * se(vw))
    assert np.all(np.abs(w.var(axis=1) - vw) < 0.1 * vw + 5 * se(vw) * 0.5)


def rw_scales(alpha):
    a = max(alpha, 0.02)
    return np.array([0.15 / a, (1 + math.sqrt(1 / a)) * 0.15, (1 + math.sqrt(1 / a)) * 0.2])


def test_init_prior_moments(orc):
    K, n = 4, 1 << 15
    cfg = orc.gmm_cfg(n, 11, K)
    pop, ll, lp = orc.gmm_init(cfg, np.array([0.0, 1.0]))
    _prior_moment_check(pop, K, n)


def test_alpha_zero_keeps_prior(orc):
    # with alpha == 0 all increments vanish: lw stays 0, log Z = 0, ESS = N,
    # no resampling, and the MCMC keeps the particles distributed as the prior
    K, n, T = 4, 1 << 14, 12
    y = synth.gmm_data_four_components(20, 5)
    cfg = orc.gmm_cfg(n, 21, K)
    alpha = np.zeros(T + 1)
    scales = np.array([rw_scales(0.0)] * (T + 1))
    logz, hist, pop, lw = orc.gmm_run(cfg, y, alpha, scales)
    assert logz == 0.0 and np.all(lw == 0.0)
    assert np.allclose(hist[1:, 0], n, rtol=1e-12, atol=0) and np.all(hist[:, 1] == 0)
    assert np.all(hist[1:, 5:8] > 0)
    _prior_moment_check(pop, K, n)


@pytest.mark.parametrize("move,scale", [("rw", (7.5, 1.2, 1.6)), ("mala", (2.5, 0.8, 0.8))])
def test_point_mass_start_reaches_prior(orc, move, scale):
    # every chain starts from the same point; under the alpha = 0 kernel the
    # population must relax to the prior (catches kernels that never move or
    # that leave the wrong distribution invariant)
    K, n, sweeps = 3, 1 << 13, 80
    y = np.array([0.3, -1.0, 2.0])
    cfg = orc.gmm_cfg(n, 31, K, move=move)
    start = np.concatenate([np.full(K, 3.0), np.full(K, 0.5), np.full(K - 1, -0.5)])
    pop = np.tile(start[:, None], (1, n))
    ll = np.full(n, orc.gmm_loglik(start, K, y))
    lp = np.full(n, orc.gmm_logprior(cfg, start))
    grad = None
    if move == "mala":
        grad = np.tile(orc.gmm_loglik(start, K, y, grad=True)[1][:, None], (1, n))
    accepted = np.zeros(3)
    for s in range(sweeps):
        for b in range(3):
            pop, ll, lp, grad, acc = orc.gmm_block(cfg, s + 1, b, 0, 0.0, scale[b], y, pop, ll, lp, grad)
            accepted[b] += acc.mean()
    assert np.all(accepted / sweeps > 0.05)
    _prior_moment_check(pop, K, n)
    # cached values stay consistent with the state
    for i in range(0, n, n // 7):
        assert ll[i] == pytest.approx(orc.gmm_loglik(pop[:, i], K, y), abs=1e-12)
        assert lp[i] == pytest.approx(orc.gmm_logprior(cfg, pop[:, i]), abs=1e-12)
        if grad is not None:
            assert np.allclose(grad[:, i], orc.gmm_loglik(pop[:, i], K, y, grad=True)[1], atol=1e-12)


@pytest.mark.parametrize("move", ["rw", "mala"])
def test_k1_evidence_matches_quadrature(orc, move):
    # one component: log p(y) by conjugacy in mu and 1-D quadrature in lambda
    y = synth.gmm_data(30, [1.0], 2.0, [1.0], 99)
    ref = gmm_k1_log_evidence(y, 0.0, 10.0, 1.0, 1.0)
    T = 40
    alpha = synth.prior_tempering(T, 4.0)
    if move == "rw":
        scales = np.array([rw_scales(a) for a in alpha])
    else:
        scales = np.array([0.5 * rw_scales(a) / 0.15 * np.array([0.15, 0.15, 0.15]) for a in alpha])
    vals = []
    for seed in range(1, 9):
        cfg = orc.gmm_cfg(1 << 12, seed, 1, move=move)
        logz, hist, _, _ = orc.gmm_run(cfg, y, alpha, scales)
        vals.append(logz)
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(vals.size)
    assert abs(vals.mean() - ref) < 4 * se + 0.02, (vals.mean(), ref, se)


def _conjugate_path(y, alpha):
    """E_alpha[log N(y | theta, 1)] under q_alpha = N(theta | 0, 1) N(y |
    theta, 1)^alpha: theta ~ N(alpha y / (1 + alpha), 1 / (1 + alpha))."""
    a = np.asarray(alpha, dtype=float)
    m = a * y / (1.0 + a)
    v = 1.0 / (1.0 + a)
    return -0.5 * math.log(2 * math.pi) - 0.5 * ((y - m) ** 2 + v)


@pytest.mark.parametrize("power", [1.0, 4.0])
def test_path_sampling_trapezoid_closed_form(orc, power):
    # Eq. path_identity on a conjugate Gaussian: log Z = log N(y | 0, 2); the
    # trapezoid of Eq. path_est converges at O(1/T^2), and since E_alpha[l]
    # increases with alpha (its derivative is a variance) the error is at
    # most half the spread between the left and right Riemann sums
    y = 1.7
    exact = stats.norm.logpdf(y, 0.0, math.sqrt(2.0))
    errs = []
    for T in (25, 50, 100, 200):
        alpha = synth.prior_tempering(T, power)
        U = _conjugate_path(y, alpha)
        ps = orc.path_sampling(alpha, U)
        bound = 0.5 * float(np.sum(np.diff(alpha) * np.diff(U)))
        assert abs(ps - exact) <= bound + 1e-14
        errs.append(abs(ps - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 3.5) & (ratios < 4.5)), ratios


def test_path_sampling_matches_direct_estimate_k1(orc):
    # the sampler's own U_t: path sampling and the direct estimate both reach
    # the quadrature evidence of a one-component model, the former up to its
    # trapezoid error (bounded as above, from the seed-averaged integrands)
    y = synth.gmm_data(30, [1.0], 2.0, [1.0], 99)
    ref = gmm_k1_log_evidence(y, 0.0, 10.0, 1.0, 1.0)
    T = 40
    alpha = synth.prior_tempering(T, 4.0)
    scales = np.array([rw_scales(a) for a in alpha])
    ps, ds, us = [], [], []
    for seed in range(1, 9):
        cfg = orc.gmm_cfg(1 << 12, seed, 1)
        logz, hist, _, _ = orc.gmm_run(cfg, y, alpha, scales)
        ds.append(logz)
        ps.append(hist[T, 9])
        us.append(hist[:, 8])
        # the recorded running value is the trapezoid of the recorded U
        assert hist[T, 9] == pytest.approx(orc.path_sampling(alpha, hist[:, 8]), abs=1e-9)
        assert np.all(np.diff(hist[:, 9][1:]) == pytest.approx(
            0.5 * np.diff(alpha)[1:] * (hist[2:, 8] + hist[1:-1, 8]), abs=1e-9))
    ps, ds = np.array(ps), np.array(ds)
    ubar = np.mean(us, axis=0)
    bound = 0.5 * float(np.sum(np.diff(alpha) * np.abs(np.diff(ubar))))
    se = ps.std(ddof=1) / math.sqrt(ps.size)
    assert abs(ps.mean() - ref) <= bound + 4 * se + 0.02, (ps.mean(), ref, bound, se)
    assert abs(ds.mean() - ref) < 4 * ds.std(ddof=1) / math.sqrt(ds.size) + 0.02


@pytest.mark.parametrize("move", ["rw", "mala"])
def test_particle_subset_equals_population_columns(orc, move):
    # the sampled-column forms used at sizes the oracle cannot replay whole:
    # particle ids pick the random numbers, so a subset reproduces exactly
    # the corresponding columns of the whole-population update
    K, n, nd = 3, 700, 50
    y = synth.gmm_data(nd, [-2.0, 0.5, 2.5], 2.0, [1, 1, 1], 9)
    cfg = orc.gmm_cfg(n, 13, K, move=move)
    pop, ll, lp = orc.gmm_init(cfg, y)
    ids = np.array([0, 3, 64, 65, 311, 699])
    p2, l2, q2 = orc.gmm_init_ids(cfg, y, ids)
    assert np.array_equal(p2, pop[:, ids]) and np.array_equal(l2, ll[ids])
    assert np.array_equal(q2, lp[ids])
    grad = None
    if move == "mala":
        grad = np.stack([orc.gmm_loglik(pop[:, i], K, y, grad=True)[1] for i in range(n)], axis=1)
    for b in range(3):
        full = orc.gmm_block_trace(cfg, 5, b, 0, 0.4, 0.1, y, pop, ll, lp, grad)
        sub = orc.gmm_block_trace_ids(cfg, 5, b, 0, 0.4, 0.1, y, ids, pop[:, ids], ll[ids],
                                      lp[ids], None if grad is None else grad[:, ids])
        for u, v in zip(full, sub):
            if u is not None:
                assert np.array_equal(u[..., ids], v)
        pop, ll, lp, grad = full[:4]


def test_run_records_decision_margins(orc):
    # the whole run's margin columns: the Metropolis margin equals the
    # smallest |log r - log u| / size over the replayed blocks, the resample
    # margin |ESS - tau N| / tau N, and no margin is recorded at step 0
    K, n, nd, T = 2, 400, 30, 4
    y = synth.gmm_data(nd, [-1.0, 2.0], 2.0, [1, 1], 4)
    alphas = np.linspace(0.0, 1.0, T + 1) ** 2
    scales = np.full((T + 1, 3), 0.2)
    cfg = orc.gmm_cfg(n, 21, K, threshold=0.9)
    _, hist, _, _ = orc.gmm_run(cfg, y, alphas, scales)
    assert hist.shape == (T + 1, 13)
    assert np.all(np.isinf(hist[0, 10:13]))
    assert np.all(hist[1:, 10] >= 0) and np.all(np.isfinite(hist[1:, 10]))
    assert np.allclose(hist[1:, 11], np.abs(hist[1:, 0] - 0.9 * n) / (0.9 * n), rtol=0, atol=1e-15)
    rs = hist[1:, 1] != 0
    assert np.all(np.isinf(hist[1:, 12][~rs]))
    assert np.all((hist[1:, 12][rs] >= 0) & (hist[1:, 12][rs] <= 0.5))
    # step 1 replayed by hand: min over the blocks of the recorded margins
    pop, ll, lp = orc.gmm_init(cfg, y)
    lw = orc.gmm_reweight(np.zeros(n), ll, alphas[1], False)
    L, _, ess = orc.normalise(lw)
    if orc.resample_flag(ess, n, 0.9):
        anc, _, _ = orc.resample("systematic", 21, 1, lw)
        pop, ll, lp = pop[:, anc], ll[anc], lp[anc]
    m = np.inf
    for b in range(3):
        before_ll, before_lp = ll.copy(), lp.copy()
        pop, ll, lp, _, acc, logr, logu = orc.gmm_block_trace(cfg, 1, b, 0, alphas[1], 0.2, y,
                                                              pop, ll, lp)
        # the size behind log r: log prior and tempered likelihood of both points
        prop_ll = np.where(acc == 1, ll, np.nan)
        ok = acc == 1
        if ok.any():
            size = (1 + np.abs(before_lp[ok]) + np.abs(lp[ok])
                    + alphas[1] * (np.abs(before_ll[ok]) + np.abs(prop_ll[ok])))
            m = min(m, float(np.min(np.abs(logr[ok] - logu[ok]) / size)))
    assert hist[1, 10] <= m
