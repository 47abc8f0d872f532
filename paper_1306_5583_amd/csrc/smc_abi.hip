// smc_abi.hip -- the extern "C" entry points of libsmc: argument validation,
// context bookkeeping and kernel launches on the caller's stream.
#include <math.h>
#include <string.h>

#include <new>
#include <algorithm>
#include <mutex>
#include <string>

#include "smc_internal.hpp"

struct smc_ctx {
    smc::Ctx c;
};

namespace smc {

// Move + weight, normalisation (with the pending monitor) and resampling of
// a one-tile tracking filter in one launch (smc_core.hip); toggles c.cur
// like the move.
hipError_t launch_pf_step_tile(Ctx &c, int32_t step, int32_t obs_index, bool gather_check,
                               bool reset_check, int32_t monitor_step, double *monitor_out,
                               int32_t force);

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

static int state_rows_of(const smc_config &cfg)
{
    if (cfg.model == SMC_MODEL_CV_TRACK)
        return 4;
    const int D = 3 * cfg.K - 1;
    return cfg.move_kind == SMC_MOVE_MALA ? 2 * D + 2 : D + 2;
}

Workspace plan_workspace(const smc_config &cfg)
{
    Workspace w{};
    const int64_t n = cfg.n;
    const int64_t ntiles = ceil_div(n, TILE);
    const int64_t gtiles = ceil_div(n + 1, TILE);
    size_t off = 0;
    w.partials = off;
    off = align256(off + sizeof(TilePartial) * (size_t)ntiles);
    w.prefix = off;
    off = align256(off + sizeof(double) * (size_t)(ntiles + 1));
    w.mon = off;
    {
        // columns: sum w and the monitored rows (the tracking state, or the
        // mixture parameters and log-likelihood)
        const int64_t cols = cfg.model == SMC_MODEL_CV_TRACK ? 5 : 3 * (int64_t)cfg.K + 1;
        const int64_t t64 = ceil_div(n, WAVE);
        int64_t words = (int64_t)MON_STRIDE * ntiles;
        if (t64 <= MON64_MAX_TILES)
            words = std::max<int64_t>(words, cols * t64);
        off = align256(off + sizeof(double) * (size_t)words);
    }
    w.counters = off;
    off = align256(off + sizeof(int32_t) * 16);
    w.cf = off;
    off = align256(off + sizeof(int32_t) * 2 * (size_t)n);
    w.cf_tiles = off;
    off = align256(off + sizeof(double) * (size_t)(4 * ntiles + 2));
    if (cfg.scheme == SMC_RS_MULTINOMIAL) {
        w.g = off;
        off = align256(off + sizeof(double) * (size_t)(n + 1));
        w.gtile = off;
        off = align256(off + sizeof(double) * (size_t)gtiles);
        w.gprefix = off;
        off = align256(off + sizeof(double) * (size_t)(gtiles + 1));
    }
    w.total = off;
    return w;
}

Workspace plan_resample_workspace(int64_t n, int32_t scheme, size_t *scalars)
{
    Workspace w{};
    const int64_t ntiles = ceil_div(n, TILE);
    const int64_t gtiles = ceil_div(n + 1, TILE);
    size_t off = 0;
    *scalars = off;
    off = align256(off + sizeof(double) * SMC_SCALARS_LEN);
    w.partials = off;
    off = align256(off + sizeof(TilePartial) * (size_t)ntiles);
    w.prefix = off;
    off = align256(off + sizeof(double) * (size_t)(ntiles + 1));
    w.counters = off;
    off = align256(off + sizeof(int32_t) * 16);
    w.mon = w.cf = w.cf_tiles = off;  // not used by the one-shot resampling
    if (scheme == SMC_RS_MULTINOMIAL) {
        w.g = off;
        off = align256(off + sizeof(double) * (size_t)(n + 1));
        w.gtile = off;
        off = align256(off + sizeof(double) * (size_t)gtiles);
        w.gprefix = off;
        off = align256(off + sizeof(double) * (size_t)(gtiles + 1));
    }
    w.total = off;
    return w;
}

Prob prob_from(const smc_config &cfg, const smc_buffers &buf, const Workspace &ws,
                      void *s0, void *s1)
{
    Prob P{};
    P.kind = cfg.model;
    P.move_kind = cfg.move_kind;
    P.elem_bytes = (cfg.model == SMC_MODEL_CV_TRACK && cfg.precision == SMC_F32_STATE) ? 4 : 8;
    P.sweeps = cfg.sweeps > 0 ? cfg.sweeps : 1;
    P.n = cfg.n;
    P.n_data = cfg.model == SMC_MODEL_CV_TRACK ? (int64_t)cfg.n_obs : cfg.n_data;
    P.ntiles = ceil_div(cfg.n, TILE);
    P.key = make_key(cfg.seed);
    P.problem_id = cfg.problem_id;
    P.K = cfg.K;
    P.scheme = cfg.scheme;
    P.threshold = cfg.threshold;
    P.mv = Motion{cfg.dt, cfg.sd_pos, cfg.sd_vel};
    if (cfg.model == SMC_MODEL_CV_TRACK) {
        const double sc = cfg.obs_scale;
        P.obs.inv_s = 1.0 / sc;
        if (isinf(cfg.obs_nu)) {
            P.obs.gaussian = 1;
            P.obs.c = -0.5 * log(2.0 * M_PI * sc * sc);
            P.obs.half_nu1 = 0.0;
            P.obs.inv_nu = 0.0;
        } else {
            const double nu = cfg.obs_nu;
            P.obs.gaussian = 0;
            P.obs.half_nu1 = 0.5 * (nu + 1.0);
            P.obs.inv_nu = 1.0 / nu;
            P.obs.c = cfg.paper_compatible_loglik ? 0.0
                                                  : lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) -
                                                        0.5 * log(nu * M_PI) - log(sc);
        }
    }
    for (int k = 0; k < 4; ++k)
        P.init_sd[k] = cfg.init_sd[k];
    if (cfg.model == SMC_MODEL_GMM_TEMPERED) {
        P.prior = GmmPrior{cfg.prior_mu_mean, 1.0 / (2.0 * cfg.prior_mu_sd * cfg.prior_mu_sd),
                           cfg.prior_gamma_shape, cfg.prior_gamma_rate, cfg.prior_dir_rho};
        P.mu_sd = cfg.prior_mu_sd;
    }
    P.state[0] = s0;
    P.state[1] = s1;
    P.lw = buf.log_weight;
    P.anc = buf.ancestors;
    P.data = buf.data;
    P.hist = buf.history;
    P.hist_len = buf.history ? buf.history_len : 0;
    P.scalars = buf.scalars;
    char *w = static_cast<char *>(buf.workspace);
    P.partials = reinterpret_cast<TilePartial *>(w + ws.partials);
    P.prefix = reinterpret_cast<double *>(w + ws.prefix);
    P.mon = reinterpret_cast<double *>(w + ws.mon);
    P.counters = reinterpret_cast<int32_t *>(w + ws.counters);
    P.sched = nullptr;
    return P;
}

Prob make_prob(const Ctx &c) { return prob_from(c.cfg, c.buf, c.ws, c.state_ptr(), c.other_ptr()); }

smc_status validate_config(const smc_config *cfg, std::string &err)
{
    if (!cfg) {
        err = "config is NULL";
        return SMC_ERR_INVALID_ARG;
    }
    if (cfg->abi_version != SMC_ABI_VERSION) {
        err = "abi_version mismatch";
        return SMC_ERR_INVALID_ARG;
    }
    if (cfg->n < 1 || cfg->n > 0x7FFFFFFFLL) {
        err = "n must be in [1, 2^31 - 1]";
        return SMC_ERR_INVALID_ARG;
    }
    if (cfg->threshold != cfg->threshold) {
        err = "threshold is NaN";
        return SMC_ERR_INVALID_ARG;
    }
    if (cfg->scheme != SMC_RS_MULTINOMIAL && cfg->scheme != SMC_RS_SYSTEMATIC &&
        cfg->scheme != SMC_RS_STRATIFIED) {
        err = "unknown resampling scheme";
        return SMC_ERR_INVALID_ARG;
    }
    if (cfg->model == SMC_MODEL_CV_TRACK) {
        if (cfg->precision != SMC_F64 && cfg->precision != SMC_F32_STATE) {
            err = "unknown precision";
            return SMC_ERR_INVALID_ARG;
        }
        if (!(cfg->obs_scale > 0.0) || !(cfg->obs_nu > 0.0) || !(cfg->sd_pos >= 0.0) ||
            !(cfg->sd_vel >= 0.0) || !isfinite(cfg->dt)) {
            err = "invalid tracking-model parameters";
            return SMC_ERR_INVALID_ARG;
        }
        if (cfg->n_obs < 1) {
            err = "n_obs must be >= 1";
            return SMC_ERR_INVALID_ARG;
        }
        for (int k = 0; k < 4; ++k)
            if (!(cfg->init_sd[k] >= 0.0)) {
                err = "init_sd must be >= 0";
                return SMC_ERR_INVALID_ARG;
            }
    } else if (cfg->model == SMC_MODEL_GMM_TEMPERED) {
        if (cfg->K < 1 || cfg->K > 16) {
            err = "K must be in [1, 16]";
            return SMC_ERR_INVALID_ARG;
        }
        if (cfg->n_data < 1) {
            err = "n_data must be >= 1";
            return SMC_ERR_INVALID_ARG;
        }
        if (cfg->precision != SMC_F64) {
            err = "the mixture sampler runs in double precision only";
            return SMC_ERR_INVALID_ARG;
        }
        if (!(cfg->prior_mu_sd > 0.0) || !(cfg->prior_gamma_shape > 0.0) ||
            !(cfg->prior_gamma_rate > 0.0) || !(cfg->prior_dir_rho > 0.0)) {
            err = "invalid prior hyper-parameters";
            return SMC_ERR_INVALID_ARG;
        }
        if (cfg->move_kind != SMC_MOVE_RW && cfg->move_kind != SMC_MOVE_MALA) {
            err = "unknown move kind";
            return SMC_ERR_INVALID_ARG;
        }
        if (cfg->sweeps < 0 || cfg->sweeps > 64) {
            err = "sweeps must be in [0, 64]";
            return SMC_ERR_INVALID_ARG;
        }
    } else {
        err = "unknown model";
        return SMC_ERR_INVALID_ARG;
    }
    return SMC_OK;
}

static bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

smc_status validate_buffers(const smc_config &cfg, const smc_buffers *b, std::string &err)
{
    if (!b) {
        err = "buffers is NULL";
        return SMC_ERR_INVALID_ARG;
    }
    const int eb = (cfg.model == SMC_MODEL_CV_TRACK && cfg.precision == SMC_F32_STATE) ? 4 : 8;
    if (!b->state || !b->state_alt || !b->log_weight || !b->ancestors || !b->data ||
        !b->workspace || !b->scalars) {
        err = "a required buffer pointer is NULL";
        return SMC_ERR_INVALID_ARG;
    }
    if (b->state == b->state_alt) {
        err = "state and state_alt must be distinct";
        return SMC_ERR_INVALID_ARG;
    }
    if (!aligned(b->state, eb) || !aligned(b->state_alt, eb) || !aligned(b->log_weight, 8) ||
        !aligned(b->ancestors, 4) || !aligned(b->data, 8) || !aligned(b->workspace, 256) ||
        !aligned(b->scalars, 8) || (b->history && !aligned(b->history, 8))) {
        err = "misaligned buffer";
        return SMC_ERR_INVALID_ARG;
    }
    const Workspace w = plan_workspace(cfg);
    if (b->workspace_bytes < w.total) {
        err = "workspace too small (" + std::to_string(b->workspace_bytes) + " < " +
              std::to_string(w.total) + ")";
        return SMC_ERR_INVALID_ARG;
    }
    if (b->history && b->history_len < 0) {
        err = "history_len < 0";
        return SMC_ERR_INVALID_ARG;
    }
    return SMC_OK;
}

smc_status device_ok(std::string &err)
{
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        (void)hipGetLastError();
        err = "no HIP device available";
        return SMC_ERR_DEVICE;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        err = "cannot query the current HIP device";
        return SMC_ERR_DEVICE;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        err = std::string("library built for gfx950, device is ") + prop.gcnArchName;
        return SMC_ERR_DEVICE;
    }
    return SMC_OK;
}

static smc_status fail(Ctx &c, smc_status s, const std::string &msg)
{
    c.last_error = msg;
    return s;
}

static smc_status hip_status(Ctx &c, hipError_t e, const char *where)
{
    if (e == hipSuccess)
        return SMC_OK;
    c.last_error = std::string(where) + ": " + hipGetErrorString(e);
    return SMC_ERR_DEVICE;
}

}  // namespace smc

using namespace smc;

extern "C" {

const char *smc_status_string(smc_status s)
{
    switch (s) {
    case SMC_OK: return "ok";
    case SMC_ERR_INVALID_ARG: return "invalid argument";
    case SMC_ERR_BAD_STATE: return "call out of order";
    case SMC_ERR_DEVICE: return "device error";
    case SMC_ERR_NUMERIC: return "numeric failure on the device";
    case SMC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

smc_status smc_state_rows(const smc_config *cfg, int32_t *rows, int32_t *elem_bytes)
{
    std::string err;
    const smc_status s = validate_config(cfg, err);
    if (s != SMC_OK)
        return s;
    if (rows)
        *rows = state_rows_of(*cfg);
    if (elem_bytes)
        *elem_bytes = (cfg->model == SMC_MODEL_CV_TRACK && cfg->precision == SMC_F32_STATE) ? 4 : 8;
    return SMC_OK;
}

smc_status smc_workspace_size(const smc_config *cfg, size_t *bytes)
{
    std::string err;
    const smc_status s = validate_config(cfg, err);
    if (s != SMC_OK)
        return s;
    if (!bytes)
        return SMC_ERR_INVALID_ARG;
    *bytes = plan_workspace(*cfg).total;
    return SMC_OK;
}

smc_status smc_create(const smc_config *cfg, const smc_buffers *buf, void *hip_stream,
                      smc_ctx **out)
{
    std::string err;
    if (!out)
        return SMC_ERR_INVALID_ARG;
    *out = nullptr;
    smc_status s = validate_config(cfg, err);
    if (s != SMC_OK)
        return s;
    s = validate_buffers(*cfg, buf, err);
    if (s != SMC_OK)
        return s;
    s = device_ok(err);
    if (s != SMC_OK)
        return s;
    smc_ctx *h = new (std::nothrow) smc_ctx();
    if (!h)
        return SMC_ERR_DEVICE;
    Ctx &c = h->c;
    c.cfg = *cfg;
    c.buf = *buf;
    c.stream = static_cast<hipStream_t>(hip_stream);
    c.ws = plan_workspace(*cfg);
    c.n = cfg->n;
    c.ntiles = ceil_div(c.n, TILE);
    c.gtiles = ceil_div(c.n + 1, TILE);
    c.state_rows = state_rows_of(*cfg);
    c.elem_bytes = (cfg->model == SMC_MODEL_CV_TRACK && cfg->precision == SMC_F32_STATE) ? 4 : 8;
    *out = h;
    return SMC_OK;
}

static void drop_profile_events(Ctx &c)
{
    for (hipEvent_t e : c.prof_ev)
        (void)hipEventDestroy(e);
    c.prof_ev.clear();
    c.prof_next = c.prof_armed = 0;
}

smc_status smc_destroy(smc_ctx *ctx)
{
    if (ctx)
        drop_profile_events(ctx->c);
    delete ctx;
    return SMC_OK;
}

smc_status smc_profile_start(smc_ctx *ctx, int32_t count)
{
    if (!ctx || count < 0 || count > (1 << 20))
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    drop_profile_events(c);
    c.prof_ev.resize(2 * (size_t)count, nullptr);
    for (int32_t k = 0; k < 2 * count; ++k) {
        // timing only: no system-scope fence at the end of the timed launch
        const hipError_t e = hipEventCreateWithFlags(&c.prof_ev[k], hipEventDisableSystemFence);
        if (e != hipSuccess) {
            c.prof_ev.resize(k);
            drop_profile_events(c);
            return fail(c, SMC_ERR_DEVICE, std::string("smc_profile_start: ") +
                                               hipGetErrorString(e));
        }
    }
    c.prof_armed = count;
    return SMC_OK;
}

smc_status smc_profile_read(smc_ctx *ctx, float *ms, int32_t capacity, int32_t *written)
{
    if (!ctx || !written || (capacity > 0 && !ms))
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    const int32_t m = c.prof_next < capacity ? c.prof_next : capacity;
    for (int32_t k = 0; k < m; ++k) {
        hipError_t e = hipEventSynchronize(c.prof_ev[2 * k + 1]);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms[k], c.prof_ev[2 * k], c.prof_ev[2 * k + 1]);
        if (e != hipSuccess)
            return fail(c, SMC_ERR_DEVICE, std::string("smc_profile_read: ") +
                                               hipGetErrorString(e));
    }
    *written = m;
    return SMC_OK;
}

smc_status smc_set_stream(smc_ctx *ctx, void *hip_stream)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    ctx->c.stream = static_cast<hipStream_t>(hip_stream);
    return SMC_OK;
}

smc_status smc_init(smc_ctx *ctx)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    c.cur = 0;
    c.armed_lw = c.armed_gather = false;
    c.last_alpha = 0.0;
    hipError_t e = launch_reset_scalars(c);
    if (e == hipSuccess)
        e = c.cfg.model == SMC_MODEL_CV_TRACK ? launch_pf_init(c) : launch_gmm_init(c);
    const smc_status s = hip_status(c, e, "smc_init");
    if (s == SMC_OK) {
        c.initialised = true;
        c.partials_valid = true;
        c.normalised = false;
    }
    return s;
}

smc_status smc_move(smc_ctx *ctx, int32_t step, const smc_move_args *args)
{
    if (!ctx || !args)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_move before smc_init");
    if (step < 0)
        return fail(c, SMC_ERR_INVALID_ARG, "step must be >= 0");
    hipError_t e;
    if (c.cfg.model == SMC_MODEL_CV_TRACK) {
        if (args->obs_index < 0 || args->obs_index >= c.cfg.n_obs)
            return fail(c, SMC_ERR_INVALID_ARG, "obs_index out of range");
        const bool fuse = args->fuse_reweight != 0;
        const bool mon = fuse && args->monitor_step >= 0;
        if (mon && !c.normalised)
            return fail(c, SMC_ERR_BAD_STATE, "a fused monitor needs normalised incoming weights");
        e = launch_pf_move(c, step, args->obs_index, fuse, c.armed_gather, fuse && c.armed_lw,
                           mon);
        if (mon) {
            c.mon_pending_step = args->monitor_step;
            c.mon_pending_rows = 4;
            c.mon_pending_out = args->monitor_out;
        }
        c.armed_gather = false;
        if (fuse) {
            c.armed_lw = false;
            c.partials_valid = true;
            c.normalised = false;
        }
    } else {
        if (!(args->alpha >= 0.0 && args->alpha <= 1.0))
            return fail(c, SMC_ERR_INVALID_ARG, "alpha must be in [0, 1]");
        for (int b = 0; b < 3; ++b)
            if (!(args->scale[b] >= 0.0) || !isfinite(args->scale[b]))
                return fail(c, SMC_ERR_INVALID_ARG, "block scales must be finite and >= 0");
        if (args->sweeps < 0 || args->sweeps > 64)
            return fail(c, SMC_ERR_INVALID_ARG, "sweeps must be in [0, 64]");
        e = launch_gmm_move(c, step, *args, c.armed_gather);
        c.armed_gather = false;
        c.last_alpha = args->alpha;
    }
    return hip_status(c, e, "smc_move");
}

smc_status smc_reweight(smc_ctx *ctx, int32_t step, const smc_reweight_args *args)
{
    (void)step;
    if (!ctx || !args)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_reweight before smc_init");
    hipError_t e;
    if (c.cfg.model == SMC_MODEL_CV_TRACK) {
        if (args->obs_index < 0 || args->obs_index >= c.cfg.n_obs)
            return fail(c, SMC_ERR_INVALID_ARG, "obs_index out of range");
        if (c.armed_gather) {
            // the weight must be evaluated at the resampled state
            e = launch_gather(c);
            if (e != hipSuccess)
                return hip_status(c, e, "smc_reweight");
            c.cur ^= 1;
            c.armed_gather = false;
        }
        e = launch_pf_reweight(c, args->obs_index, c.armed_lw);
    } else {
        if (!isfinite(args->dalpha))
            return fail(c, SMC_ERR_INVALID_ARG, "dalpha must be finite");
        if (c.armed_gather) {
            // the cached log-likelihood must be read at the resampled state
            e = launch_gather(c);
            if (e != hipSuccess)
                return hip_status(c, e, "smc_reweight");
            c.cur ^= 1;
            c.armed_gather = false;
        }
        e = launch_gmm_reweight(c, args->dalpha, c.armed_lw);
    }
    c.armed_lw = false;
    c.partials_valid = true;
    c.normalised = false;
    return hip_status(c, e, "smc_reweight");
}

smc_status smc_ess(smc_ctx *ctx, int32_t step, double *ess_host_or_null)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised || !c.partials_valid)
        return fail(c, SMC_ERR_BAD_STATE, "smc_ess needs new weights (init, move or reweight)");
    hipError_t e = launch_finalize(c, step);
    if (e == hipSuccess) {
        c.normalised = true;
        if (ess_host_or_null) {
            e = hipMemcpyAsync(ess_host_or_null, c.buf.scalars + SMC_S_ESS, sizeof(double),
                               hipMemcpyDeviceToHost, c.stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(c.stream);
        }
    }
    return hip_status(c, e, "smc_ess");
}

smc_status smc_resample(smc_ctx *ctx, int32_t step, int32_t force)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised || !c.normalised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_resample needs a normalisation (smc_ess) first");
    if (step < 0)
        return fail(c, SMC_ERR_INVALID_ARG, "step must be >= 0");
    if (c.armed_gather || c.armed_lw)
        return fail(c, SMC_ERR_BAD_STATE, "a previous resample has not been applied yet");
    const hipError_t e = launch_resample(c, step, force);
    c.armed_lw = true;
    c.armed_gather = true;
    return hip_status(c, e, "smc_resample");
}

smc_status smc_step(smc_ctx *ctx, int32_t step, const smc_move_args *args, int32_t force)
{
    if (!ctx || !args)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (c.cfg.model != SMC_MODEL_CV_TRACK)
        return fail(c, SMC_ERR_INVALID_ARG, "smc_step is the tracking filter's iteration");
    if (args->fuse_reweight == 0)
        return fail(c, SMC_ERR_INVALID_ARG, "smc_step needs the fused weight (fuse_reweight = 1)");
    const bool one_launch = c.ntiles == 1 && c.cfg.scheme != SMC_RS_MULTINOMIAL &&
                            c.mon_pending_step < 0;
    if (!one_launch) {
        smc_status s = smc_move(ctx, step, args);
        if (s == SMC_OK)
            s = smc_ess(ctx, step, nullptr);
        if (s == SMC_OK)
            s = smc_resample(ctx, step, force);
        return s;
    }
    // the checks of the three calls (the move leaves nothing pending that
    // the normalisation or the resampling would refuse)
    if (!c.initialised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_move before smc_init");
    if (step < 0)
        return fail(c, SMC_ERR_INVALID_ARG, "step must be >= 0");
    if (args->obs_index < 0 || args->obs_index >= c.cfg.n_obs)
        return fail(c, SMC_ERR_INVALID_ARG, "obs_index out of range");
    const bool mon = args->monitor_step >= 0;
    if (mon && !c.normalised)
        return fail(c, SMC_ERR_BAD_STATE, "a fused monitor needs normalised incoming weights");
    const hipError_t e =
        launch_pf_step_tile(c, step, args->obs_index, c.armed_gather, c.armed_lw,
                            mon ? args->monitor_step : -1, args->monitor_out, force);
    if (e == hipSuccess) {
        // as after smc_move, smc_ess and smc_resample
        c.partials_valid = true;
        c.normalised = true;
        c.armed_gather = true;
        c.armed_lw = true;
    }
    return hip_status(c, e, "smc_step");
}

smc_status smc_monitor(smc_ctx *ctx, int32_t step, double *out_dev)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised || !c.normalised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_monitor needs normalised weights");
    int rows;
    if (c.cfg.model == SMC_MODEL_CV_TRACK)
        rows = 4;
    else
        rows = 3 * c.cfg.K - 1 + 1;  // parameters and the log-likelihood row
    const hipError_t e = launch_monitor(c, step, out_dev, rows, c.armed_gather, c.armed_lw);
    return hip_status(c, e, "smc_monitor");
}

smc_status smc_gather(smc_ctx *ctx)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.armed_gather)
        return SMC_OK;
    const hipError_t e = launch_gather(c);
    if (e == hipSuccess) {
        c.cur ^= 1;
        c.armed_gather = false;
    }
    return hip_status(c, e, "smc_gather");
}

smc_status smc_copy_from(smc_ctx *ctx, int32_t *copy_from_dev)
{
    if (!ctx || !copy_from_dev)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    if (!c.initialised)
        return fail(c, SMC_ERR_BAD_STATE, "smc_copy_from before smc_init");
    return hip_status(c, launch_copy_from(c, copy_from_dev), "smc_copy_from");
}

smc_status smc_current_state(smc_ctx *ctx, void **state)
{
    if (!ctx || !state)
        return SMC_ERR_INVALID_ARG;
    *state = ctx->c.state_ptr();
    return SMC_OK;
}

smc_status smc_read_scalars(smc_ctx *ctx, double *host_out)
{
    if (!ctx || !host_out)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    hipError_t e = hipMemcpyAsync(host_out, c.buf.scalars, sizeof(double) * SMC_SCALARS_LEN,
                                  hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c.stream);
    return hip_status(c, e, "smc_read_scalars");
}

smc_status smc_check(smc_ctx *ctx)
{
    if (!ctx)
        return SMC_ERR_INVALID_ARG;
    Ctx &c = ctx->c;
    int32_t word = 0;
    hipError_t e = hipMemcpyAsync(&word, c.counters() + CNT_ERR, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess)
        return hip_status(c, e, "smc_check");
    if (word == 0)
        return SMC_OK;
    std::string msg = "device error word " + std::to_string(word) + ":";
    if (word & SMC_DEVERR_ZERO_WEIGHTS)
        msg += " all weights zero or non-finite at a resample;";
    if (word & SMC_DEVERR_NONFINITE)
        msg += " non-finite weight total at a normalisation;";
    if (word & SMC_DEVERR_GAMMA)
        msg += " gamma sampler exhausted its attempts;";
    c.last_error = msg;
    return SMC_ERR_NUMERIC;
}

const char *smc_last_error(const smc_ctx *ctx)
{
    if (!ctx)
        return "null context";
    return ctx->c.last_error.c_str();
}

smc_status smc_gmm_loglik_grad(const double *mu, const double *eta, const double *z, int64_t n,
                               int32_t K, const double *y, int64_t n_data, double *loglik,
                               double *grad, void *hip_stream)
{
    if (!mu || !eta || (K > 1 && !z) || !y || !loglik || n < 1 || n > 0x7FFFFFFFLL || K < 1 ||
        K > 16 || n_data < 1)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    const smc_status s = device_ok(err);
    if (s != SMC_OK)
        return s;
    const hipError_t e = launch_gmm_loglik_grad(mu, eta, z, n, K, y, n_data, loglik, grad,
                                                static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SMC_OK : SMC_ERR_DEVICE;
}

static smc_status resample_weights_args(const double *lw, int64_t n, int32_t scheme,
                                        int32_t *ancestors, double *summary)
{
    if (!lw || !ancestors || !summary || n < 1 || n > 0x7FFFFFFFLL)
        return SMC_ERR_INVALID_ARG;
    if (scheme != SMC_RS_MULTINOMIAL && scheme != SMC_RS_SYSTEMATIC &&
        scheme != SMC_RS_STRATIFIED)
        return SMC_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(lw) % 32) != 0)  // tiles load four weights at once
        return SMC_ERR_INVALID_ARG;
    return SMC_OK;
}

smc_status smc_resample_weights_workspace(int64_t n, int32_t scheme, size_t *bytes)
{
    if (!bytes || n < 1 || n > 0x7FFFFFFFLL)
        return SMC_ERR_INVALID_ARG;
    size_t sc;
    *bytes = plan_resample_workspace(n, scheme, &sc).total;
    return SMC_OK;
}

// The one-shot resampling on a workspace the caller brings (or the static
// scratch of the variant that allocates nothing): a context on the stack
// whose buffers are the caller's log-weights and ancestors and whose
// scalars, partials and counters live in the workspace.
static smc_status resample_weights_on(const double *lw, int64_t n, int32_t scheme,
                                      double threshold, int32_t force, uint64_t seed,
                                      uint32_t step, uint32_t problem, int32_t *ancestors,
                                      double *summary, char *ws, hipStream_t stream)
{
    Ctx c;
    memset(&c.cfg, 0, sizeof(c.cfg));
    c.cfg.abi_version = SMC_ABI_VERSION;
    c.cfg.model = SMC_MODEL_CV_TRACK;
    c.cfg.n = n;
    c.cfg.scheme = static_cast<smc_scheme>(scheme);
    c.cfg.threshold = threshold;
    c.cfg.seed = seed;
    c.cfg.problem_id = problem;
    c.cfg.obs_scale = 1.0;
    c.cfg.obs_nu = 1.0;
    size_t sc_off;
    c.ws = plan_resample_workspace(n, scheme, &sc_off);
    memset(&c.buf, 0, sizeof(c.buf));
    c.buf.log_weight = const_cast<double *>(lw);  // read only
    c.buf.ancestors = ancestors;
    c.buf.scalars = reinterpret_cast<double *>(ws + sc_off);
    c.buf.workspace = ws;
    c.buf.workspace_bytes = c.ws.total;
    c.stream = stream;
    c.n = n;
    c.ntiles = ceil_div(n, TILE);
    c.gtiles = ceil_div(n + 1, TILE);
    const hipError_t e = launch_resample_weights(c, (int32_t)step, force, summary);
    return e == hipSuccess ? SMC_OK : SMC_ERR_DEVICE;
}

smc_status smc_resample_weights(const double *lw, int64_t n, int32_t scheme, double threshold,
                                int32_t force, uint64_t seed, uint32_t step, uint32_t problem,
                                int32_t *ancestors, double *summary, void *workspace,
                                size_t workspace_bytes, void *hip_stream)
{
    smc_status s = resample_weights_args(lw, n, scheme, ancestors, summary);
    if (s != SMC_OK)
        return s;
    size_t sc;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % 256) != 0 ||
        workspace_bytes < plan_resample_workspace(n, scheme, &sc).total)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    if ((s = device_ok(err)) != SMC_OK)
        return s;
    return resample_weights_on(lw, n, scheme, threshold, force, seed, step, problem, ancestors,
                               summary, static_cast<char *>(workspace),
                               static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"

namespace smc {

// Workspace of smc_resample_weights_noalloc: one array per device, held
// until the process ends.  Host code never passes `scratch` itself (on the
// host it names a stand-in, not device memory): the device address comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and kernels receive that address.
static __device__ __align__(256) char scratch[SMC_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void *scratch_addr[MAX_DEVICES];

static smc_status scratch_of_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return SMC_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return SMC_ERR_DEVICE;
        }
        scratch_addr[dev] = p;
    }
    *out = scratch_addr[dev];
    return SMC_OK;
}

}  // namespace smc

extern "C" {

smc_status smc_resample_weights_noalloc(const double *lw, int64_t n, int32_t scheme,
                                        double threshold, int32_t force, uint64_t seed,
                                        uint32_t step, uint32_t problem, int32_t *ancestors,
                                        double *summary, void *hip_stream)
{
    smc_status s = resample_weights_args(lw, n, scheme, ancestors, summary);
    if (s != SMC_OK)
        return s;
    size_t sc;
    if (plan_resample_workspace(n, scheme, &sc).total > SMC_NOALLOC_SCRATCH_BYTES)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    if ((s = device_ok(err)) != SMC_OK)
        return s;
    void *ws = nullptr;
    if ((s = scratch_of_current_device(&ws)) != SMC_OK)
        return s;
    return resample_weights_on(lw, n, scheme, threshold, force, seed, step, problem, ancestors,
                               summary, static_cast<char *>(ws),
                               static_cast<hipStream_t>(hip_stream));
}

smc_status smc_draw_words(uint64_t seed, uint32_t step, uint32_t tag, uint32_t call,
                          uint32_t problem, int64_t n, uint32_t *out, void *hip_stream)
{
    if (!out || n < 1 || n > 0xFFFFFFFFLL || tag > 0xFFFFu || call > 0xFFFFu ||
        (reinterpret_cast<uintptr_t>(out) % 16) != 0)
        return SMC_ERR_INVALID_ARG;
    std::string err;
    const smc_status s = device_ok(err);
    if (s != SMC_OK)
        return s;
    const hipError_t e = launch_draw_words(seed, step, tag, call, problem, n, out,
                                           static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? SMC_OK : SMC_ERR_DEVICE;
}

}  // extern "C"
