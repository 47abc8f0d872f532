"""GPU parity of the tempered Gaussian-mixture sampler (Section 5.2) against
the oracle, through the C ABI: prior draws and the first likelihood, the
reweighting by the tempering increment, normalisation and resampling, the
three Metropolis blocks (random walk and MALA) in lock-step with every
decision checked against the oracle's log r and log u, the adjoint entry
point, a whole run end to end, and prior invariance at tempering 0."""
import math
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import (assert_ancestors, assert_close_l1, assert_gmm_run_matches,
                         decision_matches)

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


def _state(s, K):
    """(phi[D][n], ll[n], lp[n], grad or None) from the GPU state rows."""
    D = 3 * K - 1
    x = s.state().cpu().numpy()
    grad = x[D + 2:2 * D + 2] if x.shape[0] > D + 2 else None
    return x[:D].copy(), x[D].copy(), x[D + 1].copy(), None if grad is None else grad.copy()


def _mass(ll, alpha=1.0):
    # L1 mass of the log-likelihood summands: every point's log density is
    # negative for these data, so sum_k |L_k| = |l|
    return np.abs(ll) * max(alpha, 1.0) + 50.0


@pytest.mark.parametrize("K,move", [(1, "rw"), (4, "rw"), (3, "mala"), (6, "mala"),
                                    (10, "mala"), (13, "rw"), (16, "mala")])
def test_init_parity(lib, orc, K, move):
    pkg, L = lib
    n, nd = 3001, 257
    y = synth.gmm_data(nd, np.linspace(-3, 3, K), 2.0, np.ones(K), 5)
    s = pkg.GmmSampler(n, y, K, 10, seed=7, move=move)
    s.init()
    torch.cuda.synchronize()
    phi, ll, lp, grad = _state(s, K)
    ocfg = orc.gmm_cfg(n, 7, K, move=move)
    pop_o, ll_o, lp_o = orc.gmm_init(ocfg, y)
    assert_close_l1(phi, pop_o, np.abs(pop_o) + 1, 1e-12, "phi")
    assert_close_l1(ll, ll_o, _mass(ll_o), 1e-12, "loglik")
    assert_close_l1(lp, lp_o, np.abs(lp_o) + 10, 1e-12, "logprior")
    if move == "mala":
        for i in range(0, n, 97):
            _, g = orc.gmm_loglik(pop_o[:, i], K, y, grad=True)
            assert_close_l1(grad[:, i], g, np.abs(g) + 2 * nd, 1e-12, "grad %d" % i)
    assert np.all(s.log_weight.cpu().numpy() == 0.0)
    s.check()


def _lockstep_gmm(lib, orc, n, K, nd, T, move, seed=3, threshold=0.5, sweeps=1, power=4.0,
                  alpha_zero=False):
    pkg, L = lib
    _say("gmm lockstep n=%d K=%d nd=%d T=%d move=%s" % (n, K, nd, T, move))
    y, _ = synth.gmm_data_spaced(nd, K, 11)
    s = pkg.GmmSampler(n, y, K, T, seed=seed, move=move, threshold=threshold, sweeps=sweeps)
    ocfg = orc.gmm_cfg(n, seed, K, move=move, threshold=threshold, sweeps=sweeps)
    alphas = np.zeros(T + 1) if alpha_zero else synth.prior_tempering(T, power)
    s.init()
    torch.cuda.synchronize()
    a_prev = 0.0
    flips = 0
    total_decisions = 0
    for t in range(1, T + 1):
        a = float(alphas[t])
        dalpha = 0.0 if a == 0.0 else a - a_prev
        a_prev = a
        phi, ll, lp, grad = _state(s, K)
        lw_in = s.log_weight.cpu().numpy().copy()
        sc = s.scalars_host()
        reset = sc[L.SMC_S_RESAMPLED] != 0.0 and t > 1
        # reweight + normalise
        s._rargs.dalpha = dalpha
        L.smc_reweight(s.ctx, t, s._rargs)
        L.smc_ess(s.ctx, t)
        torch.cuda.synchronize()
        lw = s.log_weight.cpu().numpy()
        lw_o = orc.gmm_reweight(lw_in, ll, dalpha, reset)
        assert_close_l1(lw, lw_o, np.abs(lw_in) + np.abs(dalpha * ll) + 1, 1e-12, "lw t=%d" % t)
        sc = s.scalars_host()
        Lo, _, esso = orc.normalise(lw)
        assert abs(sc[L.SMC_S_L] - Lo) <= 1e-12 * max(1.0, abs(Lo))
        assert abs(sc[L.SMC_S_ESS] - esso) <= 1e-12 * esso
        assert decision_matches(sc[L.SMC_S_FLAG], orc.resample_flag(esso, n, threshold), esso,
                                threshold * n)
        L.smc_resample(s.ctx, t)
        torch.cuda.synchronize()
        sc = s.scalars_host()
        resampled = sc[L.SMC_S_RESAMPLED] != 0.0
        anc = s.ancestors.cpu().numpy().astype(np.int64)
        if resampled:
            anc_o, S_o, u_o = orc.resample("systematic", seed, t, lw)
            flips += assert_ancestors(anc, anc_o, S_o, u_o, what="anc t=%d" % t)
            phi, ll, lp = phi[:, anc], ll[anc], lp[anc]
            grad = None if grad is None else grad[:, anc]
        # the three blocks (one smc_move call), then the oracle replays them
        scales = pkg.rw_scales(a) if move == "rw" else pkg.mala_scales(a)
        m = L.smc_move_args()
        m.alpha = a
        for q in range(3):
            m.scale[q] = scales[q]
        L.smc_move(s.ctx, t, m)
        torch.cuda.synchronize()
        phi_g, ll_g, lp_g, grad_g = _state(s, K)
        # oracle replays the blocks from the GPU's input, carrying the GPU's
        # decisions forward where they fall in the boundary window
        po, lo_, pro, go = phi, ll, lp, grad
        margin = np.full(n, np.inf)
        for sweep in range(sweeps):
            for b in range(3):
                if b == 2 and K == 1:
                    continue
                po, lo_, pro, go, acc, logr, logu = orc.gmm_block_trace(
                    ocfg, t, b, sweep, a, scales[b], y, po, lo_, pro, go)
                margin = np.minimum(margin, np.abs(logr - logu) / np.maximum(1.0, _mass(lo_, a)))
                total_decisions += n
        # compare final states; mismatching particles must be explained by a
        # decision within the boundary window of some block
        scale_phi = np.abs(po) + np.abs(phi) + 1.0
        bad = np.zeros(n, dtype=bool)
        err = np.abs(phi_g - po) > 1e-12 * np.maximum(1.0, scale_phi)
        bad |= err.any(axis=0)
        bad |= np.abs(ll_g - lo_) > 1e-12 * _mass(lo_, a)
        if bad.any():
            idx = np.flatnonzero(bad)
            # a differing particle must have met a decision within the window
            assert np.all(margin[idx] <= 1e-11), ("t=%d: particles %s differ, margins %s"
                                                  % (t, idx[:5], margin[idx][:5]))
            flips += idx.size
        assert_close_l1(lp_g[~bad], pro[~bad], np.abs(pro[~bad]) + 10, 1e-12, "lp t=%d" % t)
        if go is not None:
            for i in np.flatnonzero(~bad)[:: max(1, n // 50)]:
                assert_close_l1(grad_g[:, i], go[:, i], np.abs(go[:, i]) + 2 * nd, 1e-12, "grad")
        L.smc_monitor(s.ctx, t)
    s.check()
    _say("  flips %d of %d decisions" % (flips, total_decisions))
    return s


@pytest.mark.parametrize("n,K,nd,move", [(2048, 4, 200, "rw"), (3000, 1, 100, "rw"),
                                         (4096, 3, 150, "mala"), (5000, 6, 300, "mala")])
def test_lockstep(lib, orc, n, K, nd, move):
    _lockstep_gmm(lib, orc, n, K, nd, 12, move)


@pytest.mark.parametrize("n,K,nd,move", [(1100, 9, 70, "mala"), (1500, 12, 50, "rw"),
                                         (1030, 16, 40, "mala")])
def test_lockstep_large_k(lib, orc, n, K, nd, move):
    # the K >= 9 kernels keep part of their state in scratch memory
    _lockstep_gmm(lib, orc, n, K, nd, 4, move)


def test_lockstep_two_sweeps(lib, orc):
    _lockstep_gmm(lib, orc, 2500, 4, 120, 6, "rw", sweeps=2)


@pytest.mark.parametrize("move", ["rw", "mala"])
def test_end_to_end_small(lib, orc, move):
    # two independent whole runs (decisions, accept counts, direct and
    # path-sampling log Z), random walk and MALA; exact decisions and 1e-12
    # agreement up to the first step whose decisions the oracle records
    # within a boundary window (none for these seeds)
    pkg, L = lib
    K, n, nd, T = (4, 4096, 100, 20) if move == "rw" else (3, 2048, 80, 12)
    y = synth.gmm_data_four_components(nd, 8)
    alphas = synth.prior_tempering(T, 4.0)
    s = pkg.GmmSampler(n, y, K, T, seed=5, move=move)
    logz_g = s.run(alphas)
    hist = s.history_host()
    f = pkg.rw_scales if move == "rw" else pkg.mala_scales
    scales = np.array([f(a) for a in alphas])
    logz_o, hist_o, pop_o, lwf_o = orc.gmm_run(orc.gmm_cfg(n, 5, K, move=move), y, alphas,
                                               scales)
    ts = assert_gmm_run_matches(hist, hist_o, alphas, L, "end-to-end %s" % move)
    _say("  compared steps 1..%d of %d" % (ts - 1, T))
    assert ts == T + 1
    assert logz_g == hist[T, L.SMC_H_LOGZ]
    assert s.log_z_path() == hist[T, L.SMC_H_PS]
    # the final population, particle by particle
    D = 3 * K - 1
    st = s.state().cpu().numpy()
    assert_close_l1(st[:D], pop_o, np.abs(pop_o) + 1.0, 1e-12, "final population")
    s.check()


@pytest.mark.parametrize("move", ["rw", "mala"])
def test_captured_run_replays_match_eager(lib, move):
    # the whole tempered run captured as one graph, replayed three times with
    # the sampler run eagerly and the host synchronised between replays:
    # every replay reproduces the eager run bit for bit (history with the
    # accept counts, both log Z estimates, final state and weights)
    pkg, L = lib
    K, n, nd, T = 3, 3000, 90, 14
    y = synth.gmm_data_four_components(nd, 8)
    alphas = synth.prior_tempering(T, 4.0)
    s = pkg.GmmSampler(n, y, K, T, seed=12, move=move)
    logz_e = s.run(alphas)
    ref = [s.history_host().copy(), s.state().cpu().numpy().copy(),
           s.log_weight.cpu().numpy().copy()]
    ps_e = s.log_z_path()
    g = s.capture_run(alphas)
    for r in range(3):
        if r == 1:
            assert s.run(alphas) == logz_e
        _say("gmm replay", r, move)
        g.replay()
        torch.cuda.synchronize()
        assert s.log_z() == logz_e
        assert s.log_z_path() == ps_e
        got = [s.history_host(), s.state().cpu().numpy(), s.log_weight.cpu().numpy()]
        for u, v in zip(got, ref):
            assert np.array_equal(u, v)
    s.check()


def test_alpha_zero_prior_invariance(lib):
    pkg, L = lib
    K, n, T = 4, 1 << 16, 15
    y = synth.gmm_data_four_components(50, 3)
    s = pkg.GmmSampler(n, y, K, T, seed=9)
    logz = s.run(np.zeros(T + 1))
    assert logz == 0.0
    hist = s.history_host()
    assert np.all(hist[1:, L.SMC_H_FLAG] == 0)
    assert np.allclose(hist[1:, L.SMC_H_ESS], n, rtol=1e-12)
    phi = s.state().cpu().numpy()[:3 * K - 1]
    mu, eta, z = phi[:K], phi[K:2 * K], phi[2 * K:]
    assert np.all(np.abs(mu.mean(axis=1)) < 5 * 10 / math.sqrt(n))
    assert np.all(np.abs(mu.var(axis=1) / 100 - 1) < 5 * math.sqrt(2 / n))
    lam = np.exp(eta)
    assert np.all(np.abs(lam.mean(axis=1) - 1) < 5 / math.sqrt(n))
    zz = np.vstack([z, np.zeros((1, n))])
    w = np.exp(zz - zz.max(axis=0)) / np.exp(zz - zz.max(axis=0)).sum(axis=0)
    assert np.all(np.abs(w.mean(axis=1) - 0.25) < 5 * math.sqrt(0.0375 / n))


@pytest.mark.parametrize("K", [1, 2, 6, 8, 11, 16])
def test_loglik_grad_entry(lib, orc, K):
    pkg, L = lib
    n, nd = 64, 10000
    y, _ = synth.gmm_data_spaced(nd, max(K, 1), 1309)
    rng = np.random.default_rng(K)
    mu = rng.normal(0, 3, (K, n))
    eta = rng.normal(0, 0.5, (K, n))
    z = rng.normal(0, 0.5, (max(K - 1, 1), n))
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    mu_d, eta_d, z_d, y_d = dev(mu), dev(eta), dev(z), dev(y)
    ll = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = torch.zeros((3 * K - 1, n), dtype=torch.float64, device="cuda")
    L.smc_gmm_loglik_grad(mu_d.data_ptr(), eta_d.data_ptr(), z_d.data_ptr(), n, K,
                          y_d.data_ptr(), nd, ll.data_ptr(), g.data_ptr(),
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    for i in range(n):
        phi = np.concatenate([mu[:, i], eta[:, i], z[:K - 1, i]])
        v, gr = orc.gmm_loglik(phi, K, y, grad=True)
        assert_close_l1(ll[i], v, abs(v) + 50, 1e-12, "ll")
        assert_close_l1(g[:, i], gr, np.abs(gr) + 2 * nd, 1e-12, "grad")


@pytest.mark.parametrize("grad", [False, True])
@pytest.mark.parametrize("K", [2, 4, 6])
def test_loglik_far_components(lib, orc, K, grad):
    # the likelihood loops take the terms' 2^x unclamped and sum a chunk
    # again with the clamp when a term is not finite: components 1e160
    # away from every point (u^2 overflows, their terms are 0) in some
    # columns, ordinary ones in the others; every value (and gradient)
    # against the oracle
    pkg, L = lib
    n, nd = 96, 1000
    y, _ = synth.gmm_data_spaced(nd, K, 2718)
    rng = np.random.default_rng(100 + K)
    mu = rng.normal(0, 3, (K, n))
    eta = rng.normal(0, 0.5, (K, n))
    z = rng.normal(0, 0.5, (K - 1, n))
    far = np.arange(n) % 3 == 0
    mu[0, far] = 1e160                 # one far component in every third column
    mu[K - 1, np.arange(n) % 6 == 1] = -1e160
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    mu_d, eta_d, z_d, y_d = dev(mu), dev(eta), dev(z), dev(y)
    ll = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = torch.zeros((3 * K - 1, n), dtype=torch.float64, device="cuda")
    L.smc_gmm_loglik_grad(mu_d.data_ptr(), eta_d.data_ptr(), z_d.data_ptr(), n, K,
                          y_d.data_ptr(), nd, ll.data_ptr(), g.data_ptr() if grad else 0,
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(ll))
    for i in range(n):
        phi = np.concatenate([mu[:, i], eta[:, i], z[:, i]])
        if grad:
            v, gr = orc.gmm_loglik(phi, K, y, grad=True)
            # the far component's log-precision derivative is a sum of
            # r (1/2 - lambda d^2 / 2) with r = 0 exactly and lambda d^2 = inf:
            # the oracle's literal product gives NaN, the limit is 0
            bad = ~np.isfinite(gr)
            assert np.all(g[bad, i] == 0.0), (i, g[bad, i])
            assert_close_l1(g[~bad, i], gr[~bad], np.abs(gr[~bad]) + 2 * nd, 1e-12, "grad")
        else:
            v = orc.gmm_loglik(phi, K, y)
        assert_close_l1(ll[i], v, abs(v) + 50, 1e-12, "ll")


def test_autograd_function_gradcheck(lib, orc):
    pkg, L = lib
    K, n, nd = 3, 8, 40
    rng = np.random.default_rng(2)
    y = torch.as_tensor(synth.gmm_data(nd, [-2.0, 0.5, 3.0], 1.5, [1, 1, 1], 4), device="cuda")
    mu = torch.tensor(rng.normal(0, 2, (K, n)), device="cuda", requires_grad=True)
    eta = torch.tensor(rng.normal(0, 0.4, (K, n)), device="cuda", requires_grad=True)
    z = torch.tensor(rng.normal(0, 0.4, (K - 1, n)), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b, c: pkg.gmm_loglik(a, b, c, y), (mu, eta, z),
                                    eps=1e-6, atol=1e-5, rtol=1e-6)
    # backward of a weighted sum equals the oracle's analytic gradient
    w = torch.tensor(rng.normal(size=n), device="cuda")
    (pkg.gmm_loglik(mu, eta, z, y) * w).sum().backward()
    yn = y.cpu().numpy()
    for i in range(n):
        phi = np.concatenate([mu[:, i].detach().cpu().numpy(), eta[:, i].detach().cpu().numpy(),
                              z[:, i].detach().cpu().numpy()])
        _, g = orc.gmm_loglik(phi, K, yn, grad=True)
        got = np.concatenate([mu.grad[:, i].cpu().numpy(), eta.grad[:, i].cpu().numpy(),
                              z.grad[:, i].cpu().numpy()])
        assert_close_l1(got, g * w[i].item(), (np.abs(g) + 2 * nd) * abs(w[i].item()), 1e-12,
                        "vjp")


def test_gradient_central_differences_c3_shape(lib, orc):
    # the K = 6, n = 10^4 workload: 64 random particles, h = 1e-6
    pkg, L = lib
    K, n, nd = 6, 64, 10000
    y, _ = synth.gmm_data_spaced(nd, K, synth.DATA_SEED[3])
    yd = torch.as_tensor(y, device="cuda")
    rng = np.random.default_rng(64)
    mu = torch.tensor(rng.normal(0, 3, (K, n)), device="cuda")
    eta = torch.tensor(rng.normal(0.4, 0.3, (K, n)), device="cuda")
    z = torch.tensor(rng.normal(0, 0.5, (K - 1, n)), device="cuda")
    from paper_1306_5583_amd.autograd import loglik_and_grad
    ll, g = loglik_and_grad(mu, eta, z, yd)
    h = 1e-6
    params = [mu, eta, z]
    rows = [(p, r) for p in range(3) for r in range(params[p].shape[0])]
    for q, (p, r) in enumerate(rows):
        plus = [t.clone() for t in params]
        minus = [t.clone() for t in params]
        plus[p][r] += h
        minus[p][r] -= h
        fd = (loglik_and_grad(*plus, yd, False)[0] - loglik_and_grad(*minus, yd, False)[0]) / (2 * h)
        fd, gq = fd.cpu().numpy(), g[q].cpu().numpy()
        assert np.all(np.abs(fd - gq) <= 1e-6 * np.abs(gq) + 1e-4), (p, r)


def test_lockstep_c2_full_size(lib, orc):
    # the random-walk benchmark shape (N = 2^14, K = 4, n = 1000): two steps in lock-step
    _lockstep_gmm(lib, orc, 1 << 14, 4, 1000, 2, "rw", power=1.0)


def _lockstep_gmm_sampled(lib, orc, n, K, nd, alphas, move, y, seed=4, m=1024):
    """Lock-step at a size where the oracle cannot replay every particle:
    the O(N) steps (reweight, normalisation, decision, ancestors) are
    compared for all particles; the Metropolis blocks, which act on each
    particle independently, are replayed by the oracle for m sampled
    particle columns per step (their own random numbers), and states,
    log-likelihoods, log priors, gradients and decisions are compared with
    the boundary-window rule.  The cached log-likelihoods feeding the
    reweighting are checked on the same sample."""
    pkg, L = lib
    T = len(alphas) - 1
    _say("gmm sampled lockstep n=%d K=%d nd=%d T=%d move=%s m=%d" % (n, K, nd, T, move, m))
    s = pkg.GmmSampler(n, y, K, T, seed=seed, move=move)
    ocfg = orc.gmm_cfg(n, seed, K, move=move)
    rng = np.random.default_rng(seed)
    s.init()
    torch.cuda.synchronize()
    # prior draws of a sample against the oracle's draws of the same particles
    ids = np.sort(rng.choice(n, m, replace=False))
    phi, ll, lp, grad = _state(s, K)
    po, lo_, pro = orc.gmm_init_ids(ocfg, y, ids)
    assert_close_l1(phi[:, ids], po, np.abs(po) + 1, 1e-12, "init phi")
    assert_close_l1(ll[ids], lo_, _mass(lo_), 1e-12, "init loglik")
    assert_close_l1(lp[ids], pro, np.abs(pro) + 10, 1e-12, "init logprior")
    a_prev = 0.0
    flips = 0
    for t in range(1, T + 1):
        a = float(alphas[t])
        dalpha = 0.0 if a == 0.0 else a - a_prev
        a_prev = a
        phi, ll, lp, grad = _state(s, K)
        lw_in = s.log_weight.cpu().numpy().copy()
        reset = s.scalars_host()[L.SMC_S_RESAMPLED] != 0.0 and t > 1
        # the cached log-likelihoods of a sample, recomputed by the oracle
        for i in rng.choice(n, 16, replace=False):
            v = orc.gmm_loglik(phi[:, i], K, y)
            assert abs(ll[i] - v) <= 1e-12 * (abs(v) + nd), (t, i)
        s._rargs.dalpha = dalpha
        L.smc_reweight(s.ctx, t, s._rargs)
        L.smc_ess(s.ctx, t)
        torch.cuda.synchronize()
        lw = s.log_weight.cpu().numpy()
        lw_o = orc.gmm_reweight(lw_in, ll, dalpha, reset)
        assert_close_l1(lw, lw_o, np.abs(lw_in) + np.abs(dalpha * ll) + 1, 1e-12, "lw t=%d" % t)
        sc = s.scalars_host()
        Lo, _, esso = orc.normalise(lw)
        assert abs(sc[L.SMC_S_L] - Lo) <= 1e-12 * max(1.0, abs(Lo))
        assert abs(sc[L.SMC_S_ESS] - esso) <= 1e-12 * esso
        assert decision_matches(sc[L.SMC_S_FLAG], orc.resample_flag(esso, n, 0.5), esso, 0.5 * n)
        L.smc_resample(s.ctx, t)
        torch.cuda.synchronize()
        if s.scalars_host()[L.SMC_S_RESAMPLED] != 0.0:
            anc = s.ancestors.cpu().numpy().astype(np.int64)
            anc_o, S_o, u_o = orc.resample("systematic", seed, t, lw)
            flips += assert_ancestors(anc, anc_o, S_o, u_o, what="anc t=%d" % t)
            phi, ll, lp = phi[:, anc], ll[anc], lp[anc]
            grad = None if grad is None else grad[:, anc]
        scales = pkg.rw_scales(a) if move == "rw" else pkg.mala_scales(a)
        mv = L.smc_move_args()
        mv.alpha = a
        for q in range(3):
            mv.scale[q] = scales[q]
        L.smc_move(s.ctx, t, mv)
        torch.cuda.synchronize()
        phi_g, ll_g, lp_g, grad_g = _state(s, K)
        ids = np.sort(rng.choice(n, m, replace=False))
        po, lo_, pro = phi[:, ids], ll[ids], lp[ids]
        go = None if grad is None else grad[:, ids]
        margin = np.full(m, np.inf)
        for b in range(3 if K > 1 else 2):
            po, lo_, pro, go, acc, logr, logu = orc.gmm_block_trace_ids(
                ocfg, t, b, 0, a, scales[b], y, ids, po, lo_, pro, go)
            margin = np.minimum(margin, np.abs(logr - logu) / np.maximum(1.0, _mass(lo_, a)))
        bad = (np.abs(phi_g[:, ids] - po) > 1e-12 * np.maximum(
            1.0, np.abs(po) + np.abs(phi[:, ids]) + 1.0)).any(axis=0)
        bad |= np.abs(ll_g[ids] - lo_) > 1e-12 * _mass(lo_, a)
        if bad.any():
            k = np.flatnonzero(bad)
            assert np.all(margin[k] <= 1e-11), ("t=%d: particles %s differ, margins %s"
                                                % (t, ids[k][:5], margin[k][:5]))
            flips += k.size
        ok = ~bad
        assert_close_l1(lp_g[ids][ok], pro[ok], np.abs(pro[ok]) + 10, 1e-12, "lp t=%d" % t)
        if go is not None:
            assert_close_l1(grad_g[:, ids][:, ok], go[:, ok], np.abs(go[:, ok]) + 2 * nd, 1e-12,
                            "grad t=%d" % t)
        _say("  step %d: alpha %.3g, %d sampled particles compared, min margin %.2e"
             % (t, a, m, float(margin.min())))
        L.smc_monitor(s.ctx, t)
    s.check()
    _say("  flips %d" % flips)


def test_lockstep_c3_shape_mala(lib, orc):
    """The K = 6, n = 10^4, N = 2^16 MALA workload in the launch
    configuration of its benchmark, two steps in lock-step on 1024 sampled
    particle columns per step (tempering exponents large enough that the
    likelihood drives the decisions)."""
    K, n, nd = 6, 1 << 16, 10000
    y, _ = synth.gmm_data_spaced(nd, K, synth.DATA_SEED[3])
    _lockstep_gmm_sampled(lib, orc, n, K, nd, np.array([0.0, 2e-3, 2e-2]), "mala", y)


def test_lockstep_c3_shape_rw(lib, orc):
    # the random-walk baseline of the same workload
    K, n, nd = 6, 1 << 16, 10000
    y, _ = synth.gmm_data_spaced(nd, K, synth.DATA_SEED[3])
    _lockstep_gmm_sampled(lib, orc, n, K, nd, np.array([0.0, 2e-3]), "rw", y, m=512)


@pytest.mark.parametrize("K", [3, 12, 16])
def test_monitor_all_rows_against_oracle(lib, orc, K):
    # importance-sampling estimates of every parameter row and the
    # log-likelihood (up to 3K = 48 rows for K = 16) after each step
    pkg, L = lib
    n, nd, T = 3000, 60, 3
    y, _ = synth.gmm_data_spaced(nd, K, 17)
    s = pkg.GmmSampler(n, y, K, T, seed=6)
    alphas = synth.prior_tempering(T, 1.0)
    s.init()
    D = 3 * K - 1
    for t in range(1, T + 1):
        s.step(t, float(alphas[t]))
        torch.cuda.synchronize()
        est = s.monitor_out.cpu().numpy()
        x = s.state().cpu().numpy()[:D + 1]
        lw = s.log_weight.cpu().numpy()
        if s.scalars_host()[L.SMC_S_RESAMPLED] != 0.0:
            lw = np.zeros(n)          # weights restart after a resample
        ref = orc.weighted_mean(x, lw)
        assert_close_l1(est, ref, np.abs(x).mean(axis=1) + 1.0, 1e-11, "monitor K=%d t=%d" % (K, t))
    s.check()


@pytest.mark.parametrize("move", ["mala", "rw"])
def test_adaptive_steps_match_oracle_replay(lib, orc, move):
    # block scales that follow the acceptance rates are host logic over the
    # GPU's own accept counts: the oracle, given the scales the run used,
    # reproduces the whole run (decisions exact, values within 1e-12)
    pkg, L = lib
    K, n, nd, T = 4, 3000, 120, 14
    y = synth.gmm_data_four_components(nd, 21)
    alphas = synth.prior_tempering(T, 2.0)
    s = pkg.GmmSampler(n, y, K, T, seed=31, move=move)
    s.run(alphas, adapt=True)
    used = s.scales_used
    base = np.array([(pkg.rw_scales if move == "rw" else pkg.mala_scales)(a) for a in alphas])
    assert not np.allclose(used[2:], base[2:])          # the factors moved
    hist = s.history_host()
    _, hist_o, pop_o, _ = orc.gmm_run(orc.gmm_cfg(n, 31, K, move=move), y, alphas, used)
    ts = assert_gmm_run_matches(hist, hist_o, alphas, L, "adaptive %s" % move)
    assert ts == T + 1
    # the factors follow the rule from the recorded accept counts
    ad = pkg.BlockAdapter(move)
    for t in range(1, T):
        f = ad.update(hist[t, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3], n)
        assert np.allclose(used[t + 1], base[t + 1] * f, rtol=1e-15, atol=0)
    s.check()
