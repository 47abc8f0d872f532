"""ctypes binding of libsmc.so (declarations in include/smc.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels
of the library.  Function names match the C entry points.  Loading fails
loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmc.so")

SMC_ABI_VERSION = 1

# smc_status
SMC_OK, SMC_ERR_INVALID_ARG, SMC_ERR_BAD_STATE, SMC_ERR_DEVICE, SMC_ERR_NUMERIC, \
    SMC_ERR_UNSUPPORTED = range(6)
# smc_model, smc_scheme, smc_precision, smc_move_kind
SMC_MODEL_CV_TRACK, SMC_MODEL_GMM_TEMPERED = 1, 2
SMC_RS_MULTINOMIAL, SMC_RS_SYSTEMATIC, SMC_RS_STRATIFIED = 0, 1, 2
SMC_F64, SMC_F32_STATE = 0, 1
SMC_MOVE_RW, SMC_MOVE_MALA = 0, 1
SCHEMES = {"multinomial": SMC_RS_MULTINOMIAL, "systematic": SMC_RS_SYSTEMATIC,
           "stratified": SMC_RS_STRATIFIED}

# scalar block and history layout
(SMC_S_L, SMC_S_L2, SMC_S_LOGZ, SMC_S_ESS, SMC_S_DLOGZ, SMC_S_FLAG, SMC_S_M, SMC_S_STOT,
 SMC_S_RESAMPLED, SMC_S_U, SMC_S_LPRE, SMC_S_PS_LOGZ, SMC_S_PS_U, SMC_S_PS_ALPHA) = range(14)
SMC_SCALARS_LEN = 16
(SMC_H_ESS, SMC_H_FLAG, SMC_H_DLOGZ, SMC_H_LOGZ, SMC_H_L, SMC_H_ACC0, SMC_H_ACC1, SMC_H_ACC2,
 SMC_H_PATH, SMC_H_MON) = range(10)
SMC_H_PS = 13
SMC_HIST_COLS = 16
SMC_DEVERR_ZERO_WEIGHTS, SMC_DEVERR_NONFINITE, SMC_DEVERR_GAMMA = 1, 2, 4

_i32, _i64, _u32, _u64, _d, _vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p)


class smc_config(ctypes.Structure):
    _fields_ = [("abi_version", _i32), ("model", _i32), ("precision", _i32), ("scheme", _i32),
                ("n", _i64), ("threshold", _d), ("seed", _u64), ("problem_id", _u32),
                ("paper_compatible_loglik", _i32),
                ("dt", _d), ("sd_pos", _d), ("sd_vel", _d), ("obs_scale", _d), ("obs_nu", _d),
                ("init_sd", _d * 4), ("n_obs", _i32),
                ("K", _i32), ("n_data", _i64), ("prior_mu_mean", _d), ("prior_mu_sd", _d),
                ("prior_gamma_shape", _d), ("prior_gamma_rate", _d), ("prior_dir_rho", _d),
                ("move_kind", _i32), ("sweeps", _i32)]


class smc_buffers(ctypes.Structure):
    _fields_ = [("state", _vp), ("state_alt", _vp), ("log_weight", _vp), ("ancestors", _vp),
                ("data", _vp), ("history", _vp), ("history_len", _i64), ("workspace", _vp),
                ("workspace_bytes", ctypes.c_size_t), ("scalars", _vp)]


class smc_move_args(ctypes.Structure):
    _fields_ = [("obs_index", _i32), ("fuse_reweight", _i32), ("alpha", _d), ("scale", _d * 3),
                ("sweeps", _i32), ("monitor_step", _i32), ("monitor_out", _vp)]

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        if "monitor_step" not in k:
            self.monitor_step = -1


class smc_reweight_args(ctypes.Structure):
    _fields_ = [("obs_index", _i32), ("dalpha", _d)]


class smc_batch_problem(ctypes.Structure):
    _fields_ = [("cfg", smc_config), ("buf", smc_buffers), ("schedule", _vp),
                ("schedule_len", _i32)]


class SmcError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__("%s failed: status %d (%s)%s" % (
            where, status, STATUS_NAMES.get(status, "?"), (": " + detail) if detail else ""))


STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "call out of order", 3: "device error",
                4: "numeric failure on the device", 5: "unsupported"}

_lib = None


def load() -> ctypes.CDLL:
    """Load libsmc.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsmc.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_1306_5583_amd/build.py" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    st = _i32
    P = ctypes.POINTER
    sigs = {
        "smc_status_string": (ctypes.c_char_p, [st]),
        "smc_state_rows": (st, [P(smc_config), P(_i32), P(_i32)]),
        "smc_workspace_size": (st, [P(smc_config), P(ctypes.c_size_t)]),
        "smc_create": (st, [P(smc_config), P(smc_buffers), _vp, P(_vp)]),
        "smc_destroy": (st, [_vp]),
        "smc_set_stream": (st, [_vp, _vp]),
        "smc_init": (st, [_vp]),
        "smc_move": (st, [_vp, _i32, P(smc_move_args)]),
        "smc_reweight": (st, [_vp, _i32, P(smc_reweight_args)]),
        "smc_ess": (st, [_vp, _i32, P(_d)]),
        "smc_step": (st, [_vp, _i32, P(smc_move_args), _i32]),
        "smc_resample": (st, [_vp, _i32, _i32]),
        "smc_monitor": (st, [_vp, _i32, _vp]),
        "smc_gather": (st, [_vp]),
        "smc_copy_from": (st, [_vp, _vp]),
        "smc_current_state": (st, [_vp, P(_vp)]),
        "smc_read_scalars": (st, [_vp, P(_d)]),
        "smc_check": (st, [_vp]),
        "smc_last_error": (ctypes.c_char_p, [_vp]),
        "smc_gmm_loglik_grad": (st, [_vp, _vp, _vp, _i64, _i32, _vp, _i64, _vp, _vp, _vp]),
        "smc_draw_words": (st, [_u64, _u32, _u32, _u32, _u32, _i64, _vp, _vp]),
        "smc_resample_weights_workspace": (st, [_i64, _i32, P(ctypes.c_size_t)]),
        "smc_resample_weights": (st, [_vp, _i64, _i32, _d, _i32, _u64, _u32, _u32, _vp, _vp,
                                      _vp, ctypes.c_size_t, _vp]),
        "smc_resample_weights_noalloc": (st, [_vp, _i64, _i32, _d, _i32, _u64, _u32, _u32, _vp,
                                              _vp, _vp]),
        "smc_profile_start": (st, [_vp, _i32]),
        "smc_profile_read": (st, [_vp, P(ctypes.c_float), _i32, P(_i32)]),
        "smc_batch_table_size": (st, [P(smc_batch_problem), _i32, P(ctypes.c_size_t)]),
        "smc_batch_create": (st, [P(smc_batch_problem), _i32, _vp, ctypes.c_size_t, _vp,
                                  P(_vp)]),
        "smc_batch_destroy": (st, [_vp]),
        "smc_batch_plan_queue": (st, [P(smc_batch_problem), _i32, _i32, _i32, _vp, _i64,
                                      P(_i64)]),
        "smc_batch_schedule": (st, [_vp, P(_i32)]),
        "smc_batch_set_schedule": (st, [_vp, _i32, _i32, _i32]),
        "smc_batch_autotune": (st, [_vp, _i32, ctypes.c_char_p]),
        "smc_batch_waves": (st, [_vp, _i32, P(_i32)]),
        "smc_batch_init": (st, [_vp]),
        "smc_batch_step": (st, [_vp]),
        "smc_batch_capture": (st, [_vp]),
        "smc_batch_replay": (st, [_vp]),
        "smc_batch_check": (st, [_vp, P(_i32)]),
        "smc_batch_last_error": (ctypes.c_char_p, [_vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return ["smc_status_string", "smc_state_rows", "smc_workspace_size", "smc_create",
            "smc_destroy", "smc_set_stream", "smc_init", "smc_move", "smc_reweight", "smc_ess",
            "smc_resample", "smc_step", "smc_monitor", "smc_gather", "smc_copy_from", "smc_current_state",
            "smc_read_scalars", "smc_check", "smc_last_error", "smc_gmm_loglik_grad",
            "smc_draw_words", "smc_resample_weights_workspace", "smc_resample_weights",
            "smc_resample_weights_noalloc",
            "smc_profile_start", "smc_profile_read", "smc_batch_table_size",
            "smc_batch_create", "smc_batch_destroy",
            "smc_batch_plan_queue", "smc_batch_schedule", "smc_batch_set_schedule",
            "smc_batch_autotune", "smc_batch_waves", "smc_batch_init", "smc_batch_step",
            "smc_batch_capture", "smc_batch_replay", "smc_batch_check", "smc_batch_last_error"]


def _check(status, where, ctx=None, batch=None):
    if status != SMC_OK:
        detail = ""
        if ctx is not None:
            msg = load().smc_last_error(ctx)
            detail = msg.decode() if msg else ""
        elif batch is not None:
            msg = load().smc_batch_last_error(batch)
            detail = msg.decode() if msg else ""
        raise SmcError(status, where, detail)


# --------------------------------------------------------------- wrappers ---

def make_config(model, n, *, seed=1, problem_id=0, scheme="systematic", threshold=0.5,
                precision=SMC_F64, paper_compatible=False, dt=0.1, sd_pos=0.02, sd_vel=0.5,
                obs_scale=0.1, obs_nu=10.0, init_sd=(1.0, 1.0, 1.0, 1.0), n_obs=1, K=1,
                n_data=1, prior=(0.0, 10.0, 1.0, 1.0, 1.0), move_kind=SMC_MOVE_RW, sweeps=1):
    c = smc_config()
    c.abi_version = SMC_ABI_VERSION
    c.model = model
    c.precision = precision
    c.scheme = SCHEMES.get(scheme, scheme)
    c.n = n
    c.threshold = threshold
    c.seed = seed
    c.problem_id = problem_id
    c.paper_compatible_loglik = int(paper_compatible)
    c.dt, c.sd_pos, c.sd_vel, c.obs_scale, c.obs_nu = dt, sd_pos, sd_vel, obs_scale, obs_nu
    for k in range(4):
        c.init_sd[k] = init_sd[k]
    c.n_obs = n_obs
    c.K = K
    c.n_data = n_data
    (c.prior_mu_mean, c.prior_mu_sd, c.prior_gamma_shape, c.prior_gamma_rate,
     c.prior_dir_rho) = prior
    c.move_kind = move_kind
    c.sweeps = sweeps
    return c


def smc_state_rows(cfg):
    rows, eb = _i32(), _i32()
    _check(load().smc_state_rows(ctypes.byref(cfg), ctypes.byref(rows), ctypes.byref(eb)),
           "smc_state_rows")
    return rows.value, eb.value


def smc_workspace_size(cfg):
    b = ctypes.c_size_t()
    _check(load().smc_workspace_size(ctypes.byref(cfg), ctypes.byref(b)), "smc_workspace_size")
    return b.value


def smc_create(cfg, bufs, stream_handle):
    ctx = _vp()
    _check(load().smc_create(ctypes.byref(cfg), ctypes.byref(bufs), _vp(stream_handle),
                             ctypes.byref(ctx)), "smc_create")
    return ctx


def smc_destroy(ctx):
    _check(load().smc_destroy(ctx), "smc_destroy")


def smc_set_stream(ctx, stream_handle):
    _check(load().smc_set_stream(ctx, _vp(stream_handle)), "smc_set_stream", ctx)


def smc_init(ctx):
    _check(load().smc_init(ctx), "smc_init", ctx)


def smc_move(ctx, step, args):
    _check(load().smc_move(ctx, step, ctypes.byref(args)), "smc_move", ctx)


def smc_reweight(ctx, step, args):
    _check(load().smc_reweight(ctx, step, ctypes.byref(args)), "smc_reweight", ctx)


def smc_ess(ctx, step, host=False):
    if host:
        v = _d()
        _check(load().smc_ess(ctx, step, ctypes.byref(v)), "smc_ess", ctx)
        return v.value
    _check(load().smc_ess(ctx, step, None), "smc_ess", ctx)
    return None


def smc_resample(ctx, step, force=False):
    _check(load().smc_resample(ctx, step, int(force)), "smc_resample", ctx)


def smc_step(ctx, step, args, force=False):
    _check(load().smc_step(ctx, step, ctypes.byref(args), int(force)), "smc_step", ctx)


def smc_monitor(ctx, step, out_ptr=None):
    _check(load().smc_monitor(ctx, step, _vp(out_ptr) if out_ptr else None), "smc_monitor", ctx)


def smc_gather(ctx):
    _check(load().smc_gather(ctx), "smc_gather", ctx)


def smc_copy_from(ctx, out_ptr):
    _check(load().smc_copy_from(ctx, out_ptr), "smc_copy_from", ctx)


def smc_current_state(ctx):
    p = _vp()
    _check(load().smc_current_state(ctx, ctypes.byref(p)), "smc_current_state", ctx)
    return p.value


def smc_read_scalars(ctx):
    out = (_d * SMC_SCALARS_LEN)()
    _check(load().smc_read_scalars(ctx, out), "smc_read_scalars", ctx)
    return list(out)


def smc_check(ctx):
    _check(load().smc_check(ctx), "smc_check", ctx)


def smc_gmm_loglik_grad(mu_ptr, eta_ptr, z_ptr, n, K, y_ptr, n_data, ll_ptr, grad_ptr,
                        stream_handle):
    _check(load().smc_gmm_loglik_grad(_vp(mu_ptr), _vp(eta_ptr), _vp(z_ptr), n, K, _vp(y_ptr),
                                      n_data, _vp(ll_ptr), _vp(grad_ptr) if grad_ptr else None,
                                      _vp(stream_handle)), "smc_gmm_loglik_grad")


def smc_draw_words(seed, step, tag, call, problem, n, out_ptr, stream_handle):
    _check(load().smc_draw_words(seed, step, tag, call, problem, n, _vp(out_ptr),
                                 _vp(stream_handle)), "smc_draw_words")


def smc_resample_weights_workspace(n, scheme):
    b = ctypes.c_size_t()
    _check(load().smc_resample_weights_workspace(n, scheme, ctypes.byref(b)),
           "smc_resample_weights_workspace")
    return b.value


def smc_resample_weights(lw_ptr, n, scheme, threshold, force, seed, step, problem, anc_ptr,
                         summary_ptr, ws_ptr, ws_bytes, stream_handle):
    _check(load().smc_resample_weights(_vp(lw_ptr), n, scheme, threshold, force, seed, step,
                                       problem, _vp(anc_ptr), _vp(summary_ptr), _vp(ws_ptr),
                                       ws_bytes, _vp(stream_handle)), "smc_resample_weights")


NOALLOC_SCRATCH_BYTES = 4 << 20   # SMC_NOALLOC_SCRATCH_BYTES


def smc_resample_weights_noalloc(lw_ptr, n, scheme, threshold, force, seed, step, problem,
                                 anc_ptr, summary_ptr, stream_handle):
    need = smc_resample_weights_workspace(n, scheme)
    if need > NOALLOC_SCRATCH_BYTES:
        raise SmcError(SMC_ERR_INVALID_ARG, "smc_resample_weights_noalloc",
                       "n=%d needs %d bytes of workspace, more than the library's static %d"
                       % (n, need, NOALLOC_SCRATCH_BYTES))
    _check(load().smc_resample_weights_noalloc(_vp(lw_ptr), n, scheme, threshold, force, seed,
                                               step, problem, _vp(anc_ptr), _vp(summary_ptr),
                                               _vp(stream_handle)),
           "smc_resample_weights_noalloc")


def smc_profile_start(ctx, count):
    _check(load().smc_profile_start(ctx, count), "smc_profile_start", ctx)


def smc_profile_read(ctx, capacity):
    out = (ctypes.c_float * max(capacity, 1))()
    w = _i32()
    _check(load().smc_profile_read(ctx, out, capacity, ctypes.byref(w)), "smc_profile_read", ctx)
    return list(out[:w.value])


# ------------------------------------------------------------------ batch ---

def _problem_array(probs):
    arr = (smc_batch_problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = p
    return arr


def smc_batch_table_size(probs):
    arr = _problem_array(probs)
    b = ctypes.c_size_t()
    _check(load().smc_batch_table_size(arr, len(probs), ctypes.byref(b)), "smc_batch_table_size")
    return b.value


def smc_batch_create(probs, table_ptr, table_bytes, stream_handle):
    arr = _problem_array(probs)
    h = _vp()
    _check(load().smc_batch_create(arr, len(probs), _vp(table_ptr), table_bytes,
                                   _vp(stream_handle), ctypes.byref(h)), "smc_batch_create")
    return h


def smc_batch_destroy(b):
    _check(load().smc_batch_destroy(b), "smc_batch_destroy")


def smc_batch_plan_queue(probs, order, per_item):
    """The step's work queue for these problems (no device work): an int32
    array [items][4] = kind, problem, tile, tiles in the item."""
    import numpy as np
    arr = _problem_array(probs)
    cnt = _i64()
    _check(load().smc_batch_plan_queue(arr, len(probs), order, per_item, None, 0,
                                       ctypes.byref(cnt)), "smc_batch_plan_queue")
    out = np.zeros((cnt.value, 4), dtype=np.int32)
    _check(load().smc_batch_plan_queue(arr, len(probs), order, per_item,
                                       out.ctypes.data_as(_vp), cnt.value, ctypes.byref(cnt)),
           "smc_batch_plan_queue")
    return out


def smc_batch_schedule(b):
    out = (_i32 * 5)()
    _check(load().smc_batch_schedule(b, out), "smc_batch_schedule", batch=b)
    return {"order": out[0], "per_item": out[1], "wgs_per_cu": out[2], "workgroups": out[3],
            "items": out[4]}


def smc_batch_set_schedule(b, order, per_item, wgs_per_cu):
    _check(load().smc_batch_set_schedule(b, order, per_item, wgs_per_cu),
           "smc_batch_set_schedule", batch=b)


def smc_batch_autotune(b, repeats, cache_path=None):
    _check(load().smc_batch_autotune(b, repeats, cache_path.encode() if cache_path else None),
           "smc_batch_autotune", batch=b)


def smc_batch_waves(b, K):
    w = _i32()
    _check(load().smc_batch_waves(b, K, ctypes.byref(w)), "smc_batch_waves", batch=b)
    return w.value


def smc_batch_init(b):
    _check(load().smc_batch_init(b), "smc_batch_init", batch=b)


def smc_batch_step(b):
    _check(load().smc_batch_step(b), "smc_batch_step", batch=b)


def smc_batch_capture(b):
    _check(load().smc_batch_capture(b), "smc_batch_capture", batch=b)


def smc_batch_replay(b):
    _check(load().smc_batch_replay(b), "smc_batch_replay", batch=b)


def smc_batch_check(b):
    """Returns (status, first_bad_problem) without raising."""
    bad = _i32()
    st = load().smc_batch_check(b, ctypes.byref(bad))
    return st, bad.value


INF = math.inf
