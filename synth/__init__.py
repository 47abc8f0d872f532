"""Seeded synthetic inputs shaped like the paper's two examples.

This module only produces *inputs*: observation sequences for the tracking
particle filter (Section 5.1, almost-constant-velocity model) and data sets for
the Bayesian Gaussian mixture sampler (Section 5.2.1).  It holds no part of the
Monte Carlo method itself (no weighting, normalisation, resampling or MCMC).
The paper's own data files are not available, so every workload is simulated
here with numpy's PCG64 generator; both the GPU path and the CPU oracle consume
the arrays produced here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

# --------------------------------------------------------------------------
# Tracking model (Section 5.1.1): state (x_pos, y_pos, x_vel, y_vel),
# observations (x_obs, y_obs) = position + scale * t_nu noise.
# --------------------------------------------------------------------------


@dataclasses.dataclass
class CVModel:
    """Parameters of the almost-constant-velocity tracking model.

    Defaults are the standard deviations of the tracking workloads (position
    noise sd 0.02, velocity noise sd 0.5, time step 0.1, Student-t observation
    noise with nu = 10 and scale 0.1, initial state N(0, I4)).  ``obs_nu =
    inf`` selects Gaussian observation noise (the linear-Gaussian variant).
    """

    dt: float = 0.1
    sd_pos: float = 0.02
    sd_vel: float = 0.5
    obs_scale: float = 0.1
    obs_nu: float = 10.0
    init_sd: tuple = (1.0, 1.0, 1.0, 1.0)


def pf_trajectory(T: int, seed: int, model: CVModel | None = None):
    """Simulate a hidden trajectory and its observations.

    Returns ``(x_true[T, 4], y[T, 2])`` as float64 arrays.  The state moves as
    pos_t = pos_{t-1} + dt * vel_{t-1} + sd_pos * n,  vel_t = vel_{t-1} +
    sd_vel * n  (each axis separately), and y_t = pos_t + obs_scale * e with e
    Student-t(obs_nu) (or standard normal when obs_nu is infinite).
    """
    m = model or CVModel()
    rng = np.random.default_rng(seed)
    x = np.empty((T, 4))
    x[0] = rng.standard_normal(4) * np.asarray(m.init_sd, dtype=np.float64)
    for t in range(1, T):
        n = rng.standard_normal(4)
        x[t, 0] = x[t - 1, 0] + m.dt * x[t - 1, 2] + m.sd_pos * n[0]
        x[t, 1] = x[t - 1, 1] + m.dt * x[t - 1, 3] + m.sd_pos * n[1]
        x[t, 2] = x[t - 1, 2] + m.sd_vel * n[2]
        x[t, 3] = x[t - 1, 3] + m.sd_vel * n[3]
    if math.isinf(m.obs_nu):
        e = rng.standard_normal((T, 2))
    else:
        e = rng.standard_t(m.obs_nu, size=(T, 2))
    y = x[:, :2] + m.obs_scale * e
    return x, np.ascontiguousarray(y)


# --------------------------------------------------------------------------
# Gaussian mixture data (Section 5.2.1).
# --------------------------------------------------------------------------


@dataclasses.dataclass
class GmmPrior:
    """Priors mu_j ~ N(mu_mean, mu_sd^2), lambda_j ~ Gamma(shape, rate),
    omega ~ Dirichlet(rho, ..., rho)."""

    mu_mean: float = 0.0
    mu_sd: float = 10.0
    gamma_shape: float = 1.0
    gamma_rate: float = 1.0
    dir_rho: float = 1.0


def gmm_data(n: int, means, precision, weights, seed: int) -> np.ndarray:
    """Draw ``n`` points iid from sum_j w_j N(means_j, 1/precision)."""
    rng = np.random.default_rng(seed)
    means = np.asarray(means, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    comp = rng.choice(len(means), size=n, p=w)
    prec = np.broadcast_to(np.asarray(precision, dtype=np.float64), means.shape)
    return means[comp] + rng.standard_normal(n) / np.sqrt(prec[comp])


def gmm_data_four_components(n: int = 1000, seed: int = 1308) -> np.ndarray:
    """The paper's simulated mixture: means (-3, 0, 3, 6), precision 2,
    equal weights."""
    return gmm_data(n, [-3.0, 0.0, 3.0, 6.0], 2.0, [0.25] * 4, seed)


def gmm_data_spaced(n: int, K: int, seed: int, precision: float = 1.5,
                    dir_alpha: float = 2.0):
    """K components with means evenly spaced in [-5, 5], a common precision
    and weights drawn once from Dirichlet(dir_alpha).  Returns (y, weights)."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.full(K, dir_alpha))
    means = np.linspace(-5.0, 5.0, K) if K > 1 else np.zeros(1)
    return gmm_data(n, means, precision, w, seed + 7919), w


def prior_tempering(T: int, power: float = 4.0) -> np.ndarray:
    """alpha_t = (t / T)^power for t = 0..T (the 'prior' annealing scheme)."""
    t = np.arange(T + 1, dtype=np.float64)
    return (t / T) ** power


# --------------------------------------------------------------------------
# Batched workload: many independent filters and samplers of uneven sizes.
# --------------------------------------------------------------------------


@dataclasses.dataclass
class BatchProblem:
    kind: str          # "pf" or "gmm"
    n_particles: int
    seed: int          # sampler seed
    data_seed: int
    K: int = 0         # mixture components (gmm)
    n_data: int = 0    # data points (gmm)


def batched_problems(n_pf: int = 128, n_gmm: int = 32, seed: int = 5583,
                     pf_log2_range=(10, 18), gmm_log2_range=(12, 16),
                     gmm_k_range=(2, 8), gmm_n_range=(500, 20000)) -> List[BatchProblem]:
    """Shapes of the batched workload: particle counts log-uniform, mixture
    sizes uniform, data counts log-uniform."""
    rng = np.random.default_rng(seed)
    probs: List[BatchProblem] = []
    for p in range(n_pf):
        n = int(2.0 ** rng.uniform(*pf_log2_range))
        probs.append(BatchProblem("pf", n, 1_000_000 + p, 2_000_000 + p))
    for q in range(n_gmm):
        p = n_pf + q
        K = int(rng.integers(gmm_k_range[0], gmm_k_range[1] + 1))
        nd = int(math.exp(rng.uniform(math.log(gmm_n_range[0]), math.log(gmm_n_range[1]))))
        n = int(2.0 ** rng.uniform(*gmm_log2_range))
        probs.append(BatchProblem("gmm", n, 1_000_000 + p, 2_000_000 + p, K, nd))
    return probs


# Data seeds of the five workloads (1306 + index).
DATA_SEED = {k: 1306 + k for k in range(5)}


def batched_workload(steps: int = 200, probs: List[BatchProblem] | None = None,
                     tempering_power: float = 4.0):
    """Inputs of every problem of a batched run: ``[(kind, kwargs), ...]``
    with kwargs n, seed, problem_id (the problem's index) and, for "pf",
    observations y[steps + 1][2] of the problem's own trajectory; for "gmm",
    K, data y (means spaced in [-5, 5]) and the exponents
    alphas[steps + 1] = (t / steps)^power."""
    probs = batched_problems() if probs is None else probs
    out = []
    for p, q in enumerate(probs):
        if q.kind == "pf":
            _, y = pf_trajectory(steps + 1, q.data_seed)
            out.append(("pf", dict(n=q.n_particles, y=y, seed=q.seed, problem_id=p)))
        else:
            y, _ = gmm_data_spaced(q.n_data, q.K, q.data_seed)
            out.append(("gmm", dict(n=q.n_particles, y=y, K=q.K, seed=q.seed, problem_id=p,
                                    alphas=prior_tempering(steps, tempering_power))))
    return out
