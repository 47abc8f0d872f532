// smc_internal.hpp -- host-side context and kernel launchers shared by the
// translation units of libsmc (not part of the public ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/smc.h"
#include "smc_device.hpp"

namespace smc {

// Workspace carve-up (byte offsets, 256-aligned), computed from the config.
struct Workspace {
    size_t partials;   // TilePartial[ntiles]
    size_t prefix;     // double[ntiles + 1]: cumulative-weight tile offsets
    size_t mon;        // monitor partial sums: double[MON_STRIDE * ntiles], or per
                       // 64-particle tile double[columns * n/64] when that is larger
    size_t g;          // double[n + 1]: multinomial cumulative exponentials
    size_t gtile;      // double[gtiles]: tile sums of the exponentials
    size_t gprefix;    // double[gtiles + 1]
    size_t counters;   // int32[16]: error word, accept counters
    size_t cf;         // int32[2n]: in-place copy layout (particle marks, duplicate parents)
    size_t cf_tiles;   // double[2 ntiles + 2 (ntiles + 1)]: its tile counts and offsets
    size_t total;
};

// Monitor partial columns per tile: sum w, then up to 63 weighted rows (the
// mixture's 3K - 1 parameters and its log-likelihood for K <= 16: 49).
constexpr int MON_STRIDE = 64;
// The standalone monitor uses 64-particle tiles while there are at most this
// many of them (populations up to 2^20), 1024-particle tiles beyond.
constexpr int64_t MON64_MAX_TILES = 16384;

// Observation log-density of the tracking model for both coordinates:
// Student-t with nu degrees of freedom and scale s per coordinate,
//   c - (nu+1)/2 log1p(((y-pos)/s)^2 / nu),
// or Gaussian c - ((y-pos)/s)^2 / 2 when gaussian != 0.  The two independent
// coordinates combine into one logarithm: log1p(a) + log1p(b) =
// log((1 + a)(1 + b)).
struct ObsModel {
    double c, half_nu1, inv_nu, inv_s;
    int gaussian;
    __device__ __forceinline__ double operator()(double px, double yx, double py, double yy) const
    {
        const double rx = (yx - px) * inv_s;
        const double ry = (yy - py) * inv_s;
        if (gaussian)
            return (c + c) - 0.5 * (rx * rx + ry * ry);
        const double q = fma(rx * rx, inv_nu, 1.0) * fma(ry * ry, inv_nu, 1.0);
        return (c + c) - half_nu1 * log_pos_d(q);
    }
};

struct Motion {
    double dt, sd_pos, sd_vel;
};

struct GmmPrior {
    double mu_mean, inv_2var, shape, rate, rho;
};

// Everything a kernel needs to know about one problem (one filter or one
// sampler): sizes, model constants and device pointers.  Passed by value to
// the single-problem kernels and read from a device table by the batched
// ones, so both run the same tile code.
struct Prob {
    int32_t kind;       // smc_model
    int32_t move_kind;  // GMM: smc_move_kind
    int32_t elem_bytes; // CV: bytes per state element (8, or 4 for the FP32 state)
    int32_t sweeps;     // GMM: Metropolis sweeps per step
    int64_t n;          // particles
    int64_t n_data;     // GMM data points / CV observation rows
    int64_t ntiles;     // 1024-particle tiles
    Key key;
    uint32_t problem_id;
    int32_t K;
    int32_t scheme;
    double threshold;
    Motion mv;
    ObsModel obs;
    double init_sd[4];
    GmmPrior prior;
    double mu_sd;
    void *state[2];
    double *lw;
    int32_t *anc;
    const double *data;
    double *hist;
    int64_t hist_len;
    double *scalars;
    TilePartial *partials;
    double *prefix;
    double *mon;
    int32_t *counters;
    const double *sched;  // batched GMM: [T+1][4] = alpha_t and the three block scales
};

struct Ctx {
    smc_config cfg;
    smc_buffers buf;
    hipStream_t stream = nullptr;
    Workspace ws{};
    int64_t n = 0;
    int64_t ntiles = 0;
    int64_t gtiles = 0;
    int state_rows = 0;
    int elem_bytes = 8;
    int cur = 0;              // which of state/state_alt holds the state
    bool initialised = false;
    bool partials_valid = false;  // a move/reweight wrote tile partials
    bool normalised = false;      // smc_ess ran after the last weight change
    // A resample kernel was launched and its outcome (device RESAMPLED
    // flag) has not yet been applied to the log-weights / the state.
    bool armed_lw = false;
    bool armed_gather = false;
    // Tempering exponent of the last mixture move (the path-sampling abscissa
    // of the next monitor).
    double last_alpha = 0.0;
    // Monitor partials produced by a move for an earlier step, completed by
    // the next normalisation (-1: none pending).
    int32_t mon_pending_step = -1;
    int mon_pending_rows = 0;
    double *mon_pending_out = nullptr;
    std::string last_error;
    // Dispatch-carried timing of the move kernel: pairs of events, the next
    // unused pair index and how many pairs are armed.
    std::vector<hipEvent_t> prof_ev;
    int prof_next = 0;
    int prof_armed = 0;

    // Next armed (start, stop) pair, if any.
    bool prof_take(hipEvent_t *a, hipEvent_t *b)
    {
        if (prof_next >= prof_armed)
            return false;
        *a = prof_ev[2 * prof_next];
        *b = prof_ev[2 * prof_next + 1];
        ++prof_next;
        return true;
    }

    void *state_ptr() const { return cur == 0 ? buf.state : buf.state_alt; }
    void *other_ptr() const { return cur == 0 ? buf.state_alt : buf.state; }
    char *ws_base() const { return static_cast<char *>(buf.workspace); }
    TilePartial *partials() const { return reinterpret_cast<TilePartial *>(ws_base() + ws.partials); }
    double *prefix() const { return reinterpret_cast<double *>(ws_base() + ws.prefix); }
    double *mon() const { return reinterpret_cast<double *>(ws_base() + ws.mon); }
    double *g() const { return reinterpret_cast<double *>(ws_base() + ws.g); }
    double *gtile() const { return reinterpret_cast<double *>(ws_base() + ws.gtile); }
    double *gprefix() const { return reinterpret_cast<double *>(ws_base() + ws.gprefix); }
    int32_t *counters() const { return reinterpret_cast<int32_t *>(ws_base() + ws.counters); }
    int32_t *cf_present() const { return reinterpret_cast<int32_t *>(ws_base() + ws.cf); }
    int32_t *cf_dup() const { return cf_present() + n; }
    double *cf_tiles() const { return reinterpret_cast<double *>(ws_base() + ws.cf_tiles); }
};

enum Counter : int { CNT_ERR = 0, CNT_ACC0 = 1, CNT_ACC1 = 2, CNT_ACC2 = 3 };

Workspace plan_workspace(const smc_config &cfg);
// Workspace of the one-shot resampling of n log-weights (tile partials and
// offsets, the scalar block at `scalars`, counters, multinomial staging).
Workspace plan_resample_workspace(int64_t n, int32_t scheme, size_t *scalars);

// Problem descriptor of a single-problem context (state[0] = the buffer the
// state currently lives in).
Prob make_prob(const Ctx &c);
Prob prob_from(const smc_config &cfg, const smc_buffers &buf, const Workspace &ws, void *s0,
               void *s1);
smc_status validate_config(const smc_config *cfg, std::string &err);
smc_status validate_buffers(const smc_config &cfg, const smc_buffers *b, std::string &err);
smc_status device_ok(std::string &err);

// --- core launchers (smc_core.hip) ---
hipError_t launch_reset_scalars(Ctx &c);
hipError_t launch_finalize(Ctx &c, int32_t step);
hipError_t launch_resample(Ctx &c, int32_t step, int32_t force);
hipError_t launch_monitor(Ctx &c, int32_t step, double *out_dev, int rows, bool gather_pending,
                          bool reset_pending);
hipError_t launch_gather(Ctx &c);
hipError_t launch_copy_from(Ctx &c, int32_t *out);
hipError_t launch_draw_words(uint64_t seed, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                             int64_t n, uint32_t *out, hipStream_t stream);
// Normalisation + resampling of c.buf.log_weight into c.buf.ancestors, then
// the five-value summary (one-shot resampling entry points).
hipError_t launch_resample_weights(Ctx &c, int32_t step, int32_t force, double *summary);

// --- CV model launchers (smc_pf.hip) ---
hipError_t launch_pf_init(Ctx &c);
hipError_t launch_pf_move(Ctx &c, int32_t step, int32_t obs_index, bool fuse, bool gather_check,
                          bool reset_check, bool monitor);
hipError_t launch_pf_reweight(Ctx &c, int32_t obs_index, bool reset_check);

// --- GMM launchers (smc_gmm.hip) ---
hipError_t launch_gmm_init(Ctx &c);
hipError_t launch_gmm_reweight(Ctx &c, double dalpha, bool reset_check);
hipError_t launch_gmm_move(Ctx &c, int32_t step, const smc_move_args &a, bool gather_check);
hipError_t launch_gmm_loglik_grad(const double *mu, const double *eta, const double *z,
                                  int64_t n, int32_t K, const double *y, int64_t n_data,
                                  double *loglik, double *grad, hipStream_t stream);
int gmm_waves(int64_t n, int64_t nd);

// --- batched launchers (a table of Prob and (problem, tile) maps) ---
hipError_t launch_pf_init_batch(const Prob *probs, const int2 *map, int64_t tiles, hipStream_t s);
hipError_t launch_finalize_batch(const Prob *probs, int32_t nprob, const int32_t *step,
                                 hipStream_t s);
hipError_t launch_resample_batch(const Prob *probs, const int2 *map, int64_t tiles,
                                 const int32_t *step, hipStream_t s);
hipError_t launch_reset_scalars_batch(const Prob *probs, int32_t nprob, hipStream_t s);
hipError_t launch_set_step(int32_t *step, int32_t value, int32_t add, hipStream_t s);
hipError_t launch_gmm_init_batch(const Prob *probs, const int2 *map64, int64_t tiles64, int K,
                                 int W, bool mala, hipStream_t s);
hipError_t launch_const_partials_batch(const Prob *probs, const int2 *map, int64_t tiles,
                                       hipStream_t s);

// --- persistent batched step (smc_persist.hip) ---
struct QItem;
int batch_step_blocks_per_cu();
hipError_t launch_batch_step(const Prob *probs, const QItem *queue, uint32_t nitems,
                             uint32_t nwg, uint32_t *sync, uint32_t *deps, hipStream_t s);
hipError_t launch_batch_sync_reset(uint32_t *sync, uint32_t *deps, int64_t nprob, hipStream_t s);
hipError_t launch_batch_ticket_rebase(uint32_t *sync, uint32_t old_per_step,
                                      uint32_t new_per_step, hipStream_t s);
hipError_t launch_batch_monitor0(const Prob *probs, int32_t nprob, hipStream_t s);

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace smc
