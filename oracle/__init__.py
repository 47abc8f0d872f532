"""CPU oracle of the SMC sweep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it.

The arithmetic lives in plain C (``smc_oracle.c``, strict IEEE FP64, built
with gcc -O2 -ffp-contract=off); this module only marshals numpy arrays
through ctypes.  Each wrapper names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "smc_oracle.c"), os.path.join(_HERE, "gmm_oracle.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

TAG_INIT, TAG_PF_MOVE, TAG_MH_MU, TAG_MH_ETA, TAG_MH_Z, TAG_MH_ACCEPT, TAG_RESAMPLE = range(1, 8)
RS_MULTINOMIAL, RS_SYSTEMATIC, RS_STRATIFIED = 0, 1, 2
SCHEMES = {"multinomial": RS_MULTINOMIAL, "systematic": RS_SYSTEMATIC,
           "stratified": RS_STRATIFIED}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE, no contraction)."""
    srcs = [s for s in _SRC if os.path.exists(s)]
    if not force and os.path.exists(_LIB_PATH):
        if all(os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in srcs):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint32)
_i64, _u64, _u32, _i32, _d = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double


class PfCfg(ctypes.Structure):
    _fields_ = [("n", _i64), ("seed", _u64), ("problem", _u32), ("fp32_state", _i32),
                ("paper_compatible", _i32), ("scheme", _i32), ("threshold", _d),
                ("dt", _d), ("sd_pos", _d), ("sd_vel", _d), ("obs_scale", _d), ("obs_nu", _d),
                ("init_sd", _d * 4)]


class GmmCfg(ctypes.Structure):
    _fields_ = [("n", _i64), ("seed", _u64), ("problem", _u32), ("K", _i32),
                ("scheme", _i32), ("move_kind", _i32), ("sweeps", _i32), ("threshold", _d),
                ("mu_mean", _d), ("mu_sd", _d), ("gamma_shape", _d), ("gamma_rate", _d),
                ("dir_rho", _d)]


def _declare(L):
    sig = {
        "orc_set_threads": (None, [_i32]),
        "orc_max_threads": (_i32, []),
        "orc_philox": (None, [_up, _up, _up]),
        "orc_draw_words": (None, [_u64, _u32, _u32, _u32, _u32, _u32, _up]),
        "orc_u53": (_d, [_u32, _u32]),
        "orc_u24": (ctypes.c_float, [_u32]),
        "orc_normal2": (None, [_u64, _u32, _u32, _u32, _u32, _u32, _dp]),
        "orc_normal4f": (None, [_u64, _u32, _u32, _u32, _u32, _u32, _fp]),
        "orc_gamma": (_d, [_u64, _u32, _u32, _u32, _u32, _u32, _d, _ip]),
        "orc_lse": (_d, [_dp, _i64]),
        "orc_normalise": (None, [_dp, _i64, _dp]),
        "orc_resample_flag": (_i32, [_d, _i64, _d]),
        "orc_resample_uniforms": (None, [_i32, _u64, _u32, _u32, _i64, _dp]),
        "orc_ancestors": (_i32, [_dp, _i64, _dp, _ip, _dp]),
        "orc_resample": (_i32, [_i32, _u64, _u32, _u32, _dp, _i64, _ip, _dp, _dp]),
        "orc_copy_from": (None, [_ip, _i64, _ip]),
        "orc_weighted_mean": (None, [_dp, _i64, _dp, _i64, _dp]),
        "orc_pf_obs_logdens": (_d, [ctypes.POINTER(PfCfg), _d, _d]),
        "orc_pf_init": (None, [ctypes.POINTER(PfCfg), _dp, _dp, _dp]),
        "orc_pf_move": (None, [ctypes.POINTER(PfCfg), _u32, _dp, _dp, _dp, _i32, _dp, _dp]),
        "orc_gather": (None, [_dp, _i64, _i64, _ip, _dp]),
        "orc_pf_run": (_d, [ctypes.POINTER(PfCfg), _i32, _dp, _dp, _dp, _dp]),
    }
    gmm_sig = {
        "orc_gmm_loglik": (_d, [_dp, _i32, _dp, _i64]),
        "orc_gmm_loglik_grad": (_d, [_dp, _i32, _dp, _i64, _dp]),
        "orc_gmm_logprior": (_d, [ctypes.POINTER(GmmCfg), _dp]),
        "orc_gmm_logprior_grad": (None, [ctypes.POINTER(GmmCfg), _dp, _dp]),
        "orc_gmm_init": (_i32, [ctypes.POINTER(GmmCfg), _dp, _i64, _dp, _dp, _dp]),
        "orc_gmm_reweight": (None, [_dp, _dp, _i64, _d, _i32]),
        "orc_gmm_block": (_i32, [ctypes.POINTER(GmmCfg), _u32, _i32, _i32, _d, _d, _dp, _i64,
                                 _dp, _dp, _dp, _dp, _ip]),
        "orc_gmm_block_trace": (_i32, [ctypes.POINTER(GmmCfg), _u32, _i32, _i32, _d, _d, _dp,
                                       _i64, _dp, _dp, _dp, _dp, _ip, _dp, _dp]),
        "orc_gmm_block_trace_ids": (_i32, [ctypes.POINTER(GmmCfg), _u32, _i32, _i32, _d, _d,
                                           _dp, _i64, ctypes.POINTER(_i64), _i64, _dp, _dp, _dp,
                                           _dp, _ip, _dp, _dp]),
        "orc_gmm_init_ids": (_i32, [ctypes.POINTER(GmmCfg), _dp, _i64, ctypes.POINTER(_i64), _i64,
                                    _dp, _dp, _dp]),
        "orc_gmm_run": (_d, [ctypes.POINTER(GmmCfg), _dp, _i64, _i32, _dp, _dp, _dp, _dp, _dp]),
        "orc_path_sampling": (_d, [_dp, _dp, _i64]),
    }
    for name, (res, args) in list(sig.items()) + list(gmm_sig.items()):
        if not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def set_threads(n: int) -> None:
    """Threads for the oracle's independent per-particle loops (the sums stay
    sequential in index order, so results do not depend on the count)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _d_ptr(a):
    return a.ctypes.data_as(_dp)


def _i_ptr(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ RNG ---

def philox(ctr, key):
    """Philox4x32-10 block: 4 words from a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(c.ctypes.data_as(_up), k.ctypes.data_as(_up), out.ctypes.data_as(_up))
    return out


def draw_words(seed, i, t, tag, j, p=0):
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_draw_words(seed, i, t, tag, j, p, out.ctypes.data_as(_up))
    return out


def u53(a, b):
    return lib().orc_u53(a, b)


def u24(w):
    return lib().orc_u24(w)


def normal2(seed, i, t, tag, j, p=0):
    z = np.zeros(2)
    lib().orc_normal2(seed, i, t, tag, j, p, _d_ptr(z))
    return z


def normal4f(seed, i, t, tag, j, p=0):
    z = np.zeros(4, dtype=np.float32)
    lib().orc_normal4f(seed, i, t, tag, j, p, z.ctypes.data_as(_fp))
    return z


def gamma(seed, i, t, tag, jbase, shape, p=0):
    fail = ctypes.c_int32(0)
    g = lib().orc_gamma(seed, i, t, tag, jbase, p, shape, ctypes.byref(fail))
    return g, bool(fail.value)


# -------------------------------------------------------------- weights ---

def lse(lw):
    lw = _f64(lw)
    return lib().orc_lse(_d_ptr(lw), lw.size)


def normalise(lw):
    """(L, L2, ESS) of unnormalised log-weights (Section 2.1)."""
    lw = _f64(lw)
    out = np.zeros(3)
    lib().orc_normalise(_d_ptr(lw), lw.size, _d_ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


def resample_flag(ess, n, threshold):
    return bool(lib().orc_resample_flag(ess, n, threshold))


def resample_uniforms(scheme, seed, t, n, p=0):
    u = np.zeros(n)
    lib().orc_resample_uniforms(SCHEMES.get(scheme, scheme), seed, t, p, n, _d_ptr(u))
    return u


def ancestors(lw, u):
    """Sorted ancestors from ordered uniforms; returns (anc, S)."""
    lw = _f64(lw)
    u = _f64(u)
    anc = np.zeros(lw.size, dtype=np.int32)
    S = np.zeros(lw.size)
    rc = lib().orc_ancestors(_d_ptr(lw), lw.size, _d_ptr(u), _i_ptr(anc), _d_ptr(S))
    if rc != 0:
        raise FloatingPointError("all weights zero or non-finite")
    return anc, S


def resample(scheme, seed, t, lw, p=0):
    """Sorted ancestor vector of one resampling step; returns (anc, S, u)."""
    lw = _f64(lw)
    n = lw.size
    anc = np.zeros(n, dtype=np.int32)
    S = np.zeros(n)
    u = np.zeros(n)
    rc = lib().orc_resample(SCHEMES.get(scheme, scheme), seed, t, p, _d_ptr(lw), n,
                            _i_ptr(anc), _d_ptr(S), _d_ptr(u))
    if rc != 0:
        raise FloatingPointError("all weights zero or non-finite")
    return anc, S, u


def path_sampling(alpha, U):
    """Trapezoid of Eq. path_est over the schedule alpha[0..T] with the
    integrands U[0..T] (Section 5.2, path sampling): the sum over t of
    (alpha_t - alpha_{t-1}) (U_t + U_{t-1}) / 2."""
    a = _f64(alpha)
    u = _f64(U)
    return float(lib().orc_path_sampling(_d_ptr(a), _d_ptr(u), a.size))


def copy_from(anc):
    anc = np.ascontiguousarray(anc, dtype=np.int32)
    out = np.zeros_like(anc)
    lib().orc_copy_from(_i_ptr(anc), anc.size, _i_ptr(out))
    return out


def weighted_mean(x, lw):
    """Importance-sampling estimate sum_i W_i x[:, i] for SoA x[dim][n]."""
    x = _f64(x)
    lw = _f64(lw)
    est = np.zeros(x.shape[0])
    lib().orc_weighted_mean(_d_ptr(x), x.shape[0], _d_ptr(lw), lw.size, _d_ptr(est))
    return est


def gather(x, anc):
    x = _f64(x)
    anc = np.ascontiguousarray(anc, dtype=np.int32)
    out = np.zeros_like(x)
    lib().orc_gather(_d_ptr(x), x.shape[0], x.shape[1], _i_ptr(anc), _d_ptr(out))
    return out


# ------------------------------------------------------ particle filter ---

def pf_cfg(n, seed, *, problem=0, fp32_state=False, paper_compatible=False,
           scheme="systematic", threshold=0.5, dt=0.1, sd_pos=0.02, sd_vel=0.5,
           obs_scale=0.1, obs_nu=10.0, init_sd=(1.0, 1.0, 1.0, 1.0)):
    c = PfCfg()
    c.n, c.seed, c.problem = n, seed, problem
    c.fp32_state, c.paper_compatible = int(fp32_state), int(paper_compatible)
    c.scheme, c.threshold = SCHEMES.get(scheme, scheme), threshold
    c.dt, c.sd_pos, c.sd_vel, c.obs_scale, c.obs_nu = dt, sd_pos, sd_vel, obs_scale, obs_nu
    for k in range(4):
        c.init_sd[k] = init_sd[k]
    return c


def pf_obs_logdens(cfg, pos, y):
    return lib().orc_pf_obs_logdens(ctypes.byref(cfg), pos, y)


def pf_init(cfg, y0):
    y0 = _f64(y0)
    x = np.zeros((4, cfg.n))
    lw = np.zeros(cfg.n)
    lib().orc_pf_init(ctypes.byref(cfg), _d_ptr(y0), _d_ptr(x), _d_ptr(lw))
    return x, lw


def pf_move(cfg, t, yt, x, lw, lw_reset):
    """One move + reweight of Algorithm 'pf' on an already-gathered population."""
    yt = _f64(yt)
    x = _f64(x)
    lw = _f64(lw)
    xo = np.zeros_like(x)
    lwo = np.zeros_like(lw)
    lib().orc_pf_move(ctypes.byref(cfg), t, _d_ptr(yt), _d_ptr(x), _d_ptr(lw), int(lw_reset),
                      _d_ptr(xo), _d_ptr(lwo))
    return xo, lwo


def pf_run(cfg, y, T=None):
    """Whole filter; returns (logZ, hist[T][9], x_final, lw_final).

    hist columns: ESS, resampled, dlogZ, logZ, L, E[x_pos], E[y_pos],
    E[x_vel], E[y_vel]."""
    y = _f64(y)
    T = y.shape[0] if T is None else T
    hist = np.zeros((T, 9))
    xf = np.zeros((4, cfg.n))
    lwf = np.zeros(cfg.n)
    logz = lib().orc_pf_run(ctypes.byref(cfg), T, _d_ptr(y), _d_ptr(hist), _d_ptr(xf), _d_ptr(lwf))
    return logz, hist, xf, lwf


# ---------------------------------------------------------- GMM sampler ---

MOVE_RW, MOVE_MALA = 0, 1


def gmm_cfg(n, seed, K, *, problem=0, scheme="systematic", move="rw", sweeps=1,
            threshold=0.5, mu_mean=0.0, mu_sd=10.0, gamma_shape=1.0, gamma_rate=1.0,
            dir_rho=1.0):
    c = GmmCfg()
    c.n, c.seed, c.problem, c.K = n, seed, problem, K
    c.scheme = SCHEMES.get(scheme, scheme)
    c.move_kind = {"rw": MOVE_RW, "mala": MOVE_MALA}.get(move, move)
    c.sweeps, c.threshold = sweeps, threshold
    c.mu_mean, c.mu_sd, c.gamma_shape, c.gamma_rate, c.dir_rho = (
        mu_mean, mu_sd, gamma_shape, gamma_rate, dir_rho)
    return c


def gmm_loglik(phi, K, y, grad=False):
    """Mixture log-likelihood of one particle phi[3K-1] (Section 5.2.1);
    with grad=True also returns dl/dphi."""
    phi = _f64(phi)
    y = _f64(y)
    if grad:
        g = np.zeros(3 * K - 1)
        v = lib().orc_gmm_loglik_grad(_d_ptr(phi), K, _d_ptr(y), y.size, _d_ptr(g))
        return v, g
    return lib().orc_gmm_loglik(_d_ptr(phi), K, _d_ptr(y), y.size)


def gmm_logprior(cfg, phi, grad=False):
    phi = _f64(phi)
    v = lib().orc_gmm_logprior(ctypes.byref(cfg), _d_ptr(phi))
    if grad:
        g = np.zeros(3 * cfg.K - 1)
        lib().orc_gmm_logprior_grad(ctypes.byref(cfg), _d_ptr(phi), _d_ptr(g))
        return v, g
    return v


def gmm_init(cfg, y):
    """Prior draws of Algorithm 'gmm'; returns (pop[3K-1][n], ll[n], lp[n])."""
    y = _f64(y)
    D = 3 * cfg.K - 1
    pop = np.zeros((D, cfg.n))
    ll = np.zeros(cfg.n)
    lp = np.zeros(cfg.n)
    fails = lib().orc_gmm_init(ctypes.byref(cfg), _d_ptr(y), y.size, _d_ptr(pop), _d_ptr(ll),
                               _d_ptr(lp))
    if fails:
        raise FloatingPointError("gamma sampler exhausted its attempts")
    return pop, ll, lp


def gmm_reweight(lw, ll, dalpha, lw_reset):
    lw = _f64(lw).copy()
    ll = _f64(ll)
    lib().orc_gmm_reweight(_d_ptr(lw), _d_ptr(ll), lw.size, dalpha, int(lw_reset))
    return lw


def gmm_block(cfg, t, block, sweep, alpha, scale, y, pop, ll, lp, grad=None):
    """One Metropolis block update (in place on copies); returns
    (pop, ll, lp, grad, accepted[n])."""
    y = _f64(y)
    pop = _f64(pop).copy()
    ll = _f64(ll).copy()
    lp = _f64(lp).copy()
    grad = None if grad is None else _f64(grad).copy()
    acc = np.zeros(cfg.n, dtype=np.int32)
    lib().orc_gmm_block(ctypes.byref(cfg), t, block, sweep, alpha, scale, _d_ptr(y), y.size,
                        _d_ptr(pop), _d_ptr(ll), _d_ptr(lp),
                        None if grad is None else _d_ptr(grad), _i_ptr(acc))
    return pop, ll, lp, grad, acc


def gmm_block_trace(cfg, t, block, sweep, alpha, scale, y, pop, ll, lp, grad=None):
    """gmm_block that also returns log r and log u of every decision."""
    y = _f64(y)
    pop = _f64(pop).copy()
    ll = _f64(ll).copy()
    lp = _f64(lp).copy()
    grad = None if grad is None else _f64(grad).copy()
    acc = np.zeros(cfg.n, dtype=np.int32)
    logr = np.zeros(cfg.n)
    logu = np.zeros(cfg.n)
    lib().orc_gmm_block_trace(ctypes.byref(cfg), t, block, sweep, alpha, scale, _d_ptr(y), y.size,
                              _d_ptr(pop), _d_ptr(ll), _d_ptr(lp),
                              None if grad is None else _d_ptr(grad), _i_ptr(acc), _d_ptr(logr),
                              _d_ptr(logu))
    return pop, ll, lp, grad, acc, logr, logu


def _ids(ids):
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    return ids, ids.ctypes.data_as(ctypes.POINTER(_i64))


def gmm_init_ids(cfg, y, ids):
    """gmm_init for the particles `ids` only: (pop[D][m], ll[m], lp[m]),
    column q being particle ids[q]."""
    y = _f64(y)
    ids, pids = _ids(ids)
    m = ids.size
    D = 3 * cfg.K - 1
    pop = np.zeros((D, m))
    ll = np.zeros(m)
    lp = np.zeros(m)
    lib().orc_gmm_init_ids(ctypes.byref(cfg), _d_ptr(y), y.size, pids, m, _d_ptr(pop),
                           _d_ptr(ll), _d_ptr(lp))
    return pop, ll, lp


def gmm_block_trace_ids(cfg, t, block, sweep, alpha, scale, y, ids, pop, ll, lp, grad=None):
    """gmm_block_trace for the particles `ids` only (columns of pop, ll, lp,
    grad in the order of ids): the Metropolis blocks act on each particle
    independently, so a sample of columns can be checked on its own."""
    y = _f64(y)
    ids, pids = _ids(ids)
    m = ids.size
    pop = _f64(pop).copy()
    ll = _f64(ll).copy()
    lp = _f64(lp).copy()
    grad = None if grad is None else _f64(grad).copy()
    acc = np.zeros(m, dtype=np.int32)
    logr = np.zeros(m)
    logu = np.zeros(m)
    lib().orc_gmm_block_trace_ids(ctypes.byref(cfg), t, block, sweep, alpha, scale, _d_ptr(y),
                                  y.size, pids, m, _d_ptr(pop), _d_ptr(ll), _d_ptr(lp),
                                  None if grad is None else _d_ptr(grad), _i_ptr(acc),
                                  _d_ptr(logr), _d_ptr(logu))
    return pop, ll, lp, grad, acc, logr, logu


def gmm_run(cfg, y, alpha, scales):
    """Whole sampler (Algorithm "gmm"); returns (logZ, hist[T+1][13],
    pop_final, lw_final).

    hist columns: ESS, resampled, dlogZ, logZ (Eq. smc-ds), L,
    accepts(mu, eta, z), U_t (Eq. path_import), the running path-sampling
    estimate (Eq. path_est), and the step's decision margins: Metropolis
    (|log r - log u| over the size of log r's terms), resampling decision
    (|ESS - tau N| / tau N) and ancestors (distance of u_i S from the nearer
    bracketing cumulative weight, over S)."""
    y = _f64(y)
    alpha = _f64(alpha)
    T = alpha.size - 1
    scales = _f64(scales).reshape(T + 1, 3)
    hist = np.zeros((T + 1, 13))
    D = 3 * cfg.K - 1
    pop = np.zeros((D, cfg.n))
    lwf = np.zeros(cfg.n)
    logz = lib().orc_gmm_run(ctypes.byref(cfg), _d_ptr(y), y.size, T, _d_ptr(alpha),
                             _d_ptr(scales), _d_ptr(hist), _d_ptr(pop), _d_ptr(lwf))
    return logz, hist, pop, lwf


# ------------------------------------------------- batch draws (checks) ---

def fill_normals(seed, t, tag, j, n, p=0):
    out = np.zeros(2 * n)
    lib().orc_fill_normals(_u64(seed), _u32(t), _u32(tag), _u32(j), _u32(p), _i64(n), _d_ptr(out))
    return out


def fill_normals_f32(seed, t, tag, j, n, p=0):
    out = np.zeros(4 * n, dtype=np.float32)
    lib().orc_fill_normals_f32(_u64(seed), _u32(t), _u32(tag), _u32(j), _u32(p), _i64(n),
                               out.ctypes.data_as(_fp))
    return out


def fill_gamma(seed, t, tag, jbase, shape, n, p=0):
    out = np.zeros(n)
    fails = ctypes.c_int32(0)
    lib().orc_fill_gamma(_u64(seed), _u32(t), _u32(tag), _u32(jbase), _u32(p), _d(shape),
                         _i64(n), _d_ptr(out), ctypes.byref(fails))
    return out, fails.value
