// smc_internal.hpp -- host-side context and kernel launchers shared by the
// translation units of libsmc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/smc.h"
#include "smc_device.hpp"

namespace smc {

// Workspace carve-up (byte offsets, 256-aligned), computed from the config.
struct Workspace {
    size_t partials;   // TilePartial[ntiles]
    size_t prefix;     // double[ntiles + 1]: cumulative-weight tile offsets
    size_t mon;        // double[ntiles * MON_STRIDE]: monitor partial sums
    size_t g;          // double[n + 1]: multinomial cumulative exponentials
    size_t gtile;      // double[gtiles]: tile sums of the exponentials
    size_t gprefix;    // double[gtiles + 1]
    size_t counters;   // int32[16]: error word, accept counters
    size_t total;
};

constexpr int MON_STRIDE = 32;  // monitor partial: sum w, then up to 31 weighted rows

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
    // Monitor partials produced by a move for an earlier step, completed by
    // the next normalisation (-1: none pending).
    int32_t mon_pending_step = -1;
    int mon_pending_rows = 0;
    double *mon_pending_out = nullptr;
    // Student-t / Gaussian observation constants (CV).
    double obs_const = 0.0;
    double obs_half_nu1 = 0.0;
    double obs_inv_scale = 0.0;
    std::string last_error;

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
};

enum Counter : int { CNT_ERR = 0, CNT_ACC0 = 1, CNT_ACC1 = 2, CNT_ACC2 = 3 };

Workspace plan_workspace(const smc_config &cfg);

// --- core launchers (smc_core.hip) ---
hipError_t launch_reset_scalars(Ctx &c);
hipError_t launch_finalize(Ctx &c, int32_t step);
hipError_t launch_resample(Ctx &c, int32_t step, int32_t force);
hipError_t launch_monitor(Ctx &c, int32_t step, double *out_dev, int rows, bool gather_pending,
                          bool reset_pending);
hipError_t launch_gather(Ctx &c);
hipError_t launch_draw_words(uint64_t seed, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                             int64_t n, uint32_t *out, hipStream_t stream);

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

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace smc
