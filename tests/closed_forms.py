"""Independent closed forms used to pin the oracle (test helpers only).

Nothing here shares arithmetic with the oracle: each function is a textbook
result written out directly (Kalman filter, Gaussian conjugacy, brute-force
allocation sums) so that a mistake in the oracle shows up as a mismatch.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, special, stats


def kalman_loglik(y, dt, sd_pos, sd_vel, obs_sd, init_sd):
    """Exact log p(y_0..y_{T-1}) and filtered means of the linear-Gaussian
    constant-velocity model (state order x_pos, y_pos, x_vel, y_vel)."""
    A = np.eye(4)
    A[0, 2] = dt
    A[1, 3] = dt
    Q = np.diag([sd_pos ** 2, sd_pos ** 2, sd_vel ** 2, sd_vel ** 2])
    B = np.zeros((2, 4))
    B[0, 0] = B[1, 1] = 1.0
    R = np.eye(2) * obs_sd ** 2
    m = np.zeros(4)
    P = np.diag(np.asarray(init_sd, dtype=float) ** 2)
    ll = 0.0
    means = []
    for t in range(y.shape[0]):
        if t > 0:
            m = A @ m
            P = A @ P @ A.T + Q
        S = B @ P @ B.T + R
        r = y[t] - B @ m
        ll += stats.multivariate_normal(mean=np.zeros(2), cov=S).logpdf(r)
        Kg = P @ B.T @ np.linalg.inv(S)
        m = m + Kg @ r
        P = (np.eye(4) - Kg @ B) @ P
        means.append(m.copy())
    return ll, np.array(means)


def gmm_loglik_bruteforce(y, mu, lam, w):
    """log of sum over all K^n allocations z of prod_k w_{z_k} N(y_k|mu_{z_k},
    1/lam_{z_k}) -- the mixture likelihood expanded term by term."""
    K = len(mu)
    terms = []
    for z in itertools.product(range(K), repeat=len(y)):
        t = 0.0
        for k, j in enumerate(z):
            t += math.log(w[j]) + stats.norm.logpdf(y[k], loc=mu[j], scale=1.0 / math.sqrt(lam[j]))
        terms.append(t)
    return float(special.logsumexp(terms))


def gmm_k1_log_evidence(y, mu_mean, mu_sd, shape, rate):
    """log p(y) for a single Gaussian with mu ~ N(mu_mean, mu_sd^2), lambda ~
    Gamma(shape, rate): the mean integrated in closed form, lambda by 1-D
    quadrature."""
    y = np.asarray(y, dtype=float)
    n = y.size
    ybar = y.mean()
    ss = float(((y - ybar) ** 2).sum())

    def log_integrand(lam):
        # prod_k N(y_k|mu,1/lam) N(mu|m0,s0^2) integrated over mu
        v = mu_sd ** 2 + 1.0 / (n * lam)
        out = 0.5 * n * math.log(lam / (2 * math.pi)) - 0.5 * lam * ss
        out += 0.5 * math.log(2 * math.pi / (n * lam))
        out += -0.5 * math.log(2 * math.pi * v) - 0.5 * (ybar - mu_mean) ** 2 / v
        out += stats.gamma.logpdf(lam, a=shape, scale=1.0 / rate)
        return out

    # locate the mode to centre the quadrature
    grid = np.exp(np.linspace(-12, 6, 4000))
    vals = np.array([log_integrand(g) for g in grid])
    peak = vals.max()
    f = lambda lam: math.exp(log_integrand(lam) - peak) if lam > 0 else 0.0
    lo, hi = grid[max(vals.argmax() - 400, 0)], grid[min(vals.argmax() + 400, grid.size - 1)]
    main, _ = integrate.quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-12)
    left, _ = integrate.quad(f, 0, lo, limit=400)
    right, _ = integrate.quad(f, hi, np.inf, limit=400)
    return peak + math.log(main + left + right)
