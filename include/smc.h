/*
 * smc.h -- C ABI of the MI355X (gfx950) sequential Monte Carlo sweep.
 *
 * The library advances a population of N weighted particles through the
 * per-iteration sweep of sequential importance sampling and resampling
 * (Zhou, "vSMC: Parallel Sequential Monte Carlo in C++", arXiv:1306.5583,
 * Section 2): move / MCMC kernel, incremental log-weight, log-sum-exp
 * normalisation with effective sample size and normalising-constant update,
 * and resampling.  Two models are built in: the almost-constant-velocity
 * tracking filter of Section 5.1 and the tempered Bayesian Gaussian mixture
 * sampler of Section 5.2.
 *
 * Conventions
 *  - Every function returns smc_status; nothing throws or aborts across the
 *    ABI.  Argument errors are reported synchronously and leave all state
 *    untouched.  Numeric failures detected on the device (all weights zero,
 *    non-finite totals) raise a device error word reported by smc_check().
 *  - All pointers in smc_buffers are DEVICE pointers owned by the caller
 *    (typically torch tensors).  They must stay valid until smc_destroy().
 *    The library allocates no device memory of its own: scratch space is the
 *    caller's workspace, sized by smc_workspace_size().
 *  - Every call enqueues work on the context's HIP stream and returns
 *    without synchronising, except where a host output is requested
 *    (smc_ess with a host pointer, smc_check, smc_read_scalars).
 *  - Decisions (whether to resample) stay on the device, so a whole step
 *    can be captured in a HIP graph.
 *  - A context must not be used from two threads at once; different
 *    contexts are independent (the per-particle / whole-collection split of
 *    Section 4.3 of the paper).
 *  - The particle count N is fixed at creation (Section 4.1, sampler
 *    construction).
 *
 * Layout in device memory (structure of arrays, particle index fastest, so
 * the 64 lanes of a wavefront read 64 consecutive elements):
 *  - CV tracking model: state rows (x_pos, y_pos, x_vel, y_vel), each [N],
 *    double (SMC_F64) or float (SMC_F32_STATE).
 *  - GMM model (K components, D = 3K-1 unconstrained parameters):
 *    rows 0..K-1 means mu_j, rows K..2K-1 eta_j = log lambda_j, rows
 *    2K..3K-2 logits z_j = log(omega_j / omega_K), row D the cached
 *    log-likelihood, row D+1 the cached log prior, and for MALA rows
 *    D+2..2D+1 the cached likelihood gradient; all double.
 *  - log_weight [N] double: unnormalised log-weights.
 *  - ancestors [N] int32: sorted (non-decreasing) parent indices of the last
 *    resample; slot i is a child of ancestors[i] (the copy_from array of the
 *    value-collection copy in Section 4.1, in sorted order).
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMC_ABI_VERSION 1

typedef enum {
    SMC_OK = 0,
    SMC_ERR_INVALID_ARG = 1, /* a pointer, size or option is invalid */
    SMC_ERR_BAD_STATE = 2,   /* call out of order (e.g. resample before init) */
    SMC_ERR_DEVICE = 3,      /* HIP runtime error or no usable gfx950 device */
    SMC_ERR_NUMERIC = 4,     /* device error word set (see SMC_DEVERR_*) */
    SMC_ERR_UNSUPPORTED = 5  /* valid request the library does not provide */
} smc_status;

typedef enum { SMC_MODEL_CV_TRACK = 1, SMC_MODEL_GMM_TEMPERED = 2 } smc_model;

/* Resampling schemes (Section 2.1; the paper names multinomial and refers
 * to Douc et al. 2005 for the others).  All produce sorted ancestors from
 * ordered uniforms u_i in (0,1] with a_i = min{ j : S_j > u_i S } over the
 * cumulative weights S_j:
 *   MULTINOMIAL: u_(i) = G_i / G_N, G the running sum of N+1 Exp(1) draws
 *   SYSTEMATIC : u_i = (i + U) / N, one U per step
 *   STRATIFIED : u_i = (i + U_i) / N, one U_i per slot                    */
typedef enum {
    SMC_RS_MULTINOMIAL = 0,
    SMC_RS_SYSTEMATIC = 1,
    SMC_RS_STRATIFIED = 2
} smc_scheme;

typedef enum { SMC_F64 = 0, SMC_F32_STATE = 1 } smc_precision;
typedef enum { SMC_MOVE_RW = 0, SMC_MOVE_MALA = 1 } smc_move_kind;

/* Device scalar block (double[SMC_SCALARS_LEN]).  Readable at any time
 * with smc_read_scalars or by copying buffers.scalars. */
enum {
    SMC_S_L = 0,        /* log sum exp(lw) of the current weights; log N after a resample */
    SMC_S_L2 = 1,       /* log sum exp(2 lw) */
    SMC_S_LOGZ = 2,     /* running log normalising-constant estimate */
    SMC_S_ESS = 3,      /* effective sample size of the last normalisation */
    SMC_S_DLOGZ = 4,    /* increment of log Z at the last normalisation */
    SMC_S_FLAG = 5,     /* resampling decision of the last normalisation (0/1) */
    SMC_S_M = 6,        /* max lw at the last normalisation */
    SMC_S_STOT = 7,     /* sum exp(lw - M): total of the cumulative weights */
    SMC_S_RESAMPLED = 8,/* 1 when the last resample call produced new ancestors */
    SMC_S_U = 9,        /* systematic offset U of the last resample */
    SMC_S_LPRE = 10,    /* L before the last resample (diagnostic) */
    SMC_S_PS_LOGZ = 11, /* GMM: running path-sampling log Z (trapezoid over alpha) */
    SMC_S_PS_U = 12,    /* GMM: U of the last monitored step */
    SMC_S_PS_ALPHA = 13,/* GMM: alpha of the last monitored step (-1: none yet) */
    SMC_SCALARS_LEN = 16
};

/* History rows (double[history_len][SMC_HIST_COLS]); row = step. */
enum {
    SMC_H_ESS = 0,
    SMC_H_FLAG = 1,
    SMC_H_DLOGZ = 2,
    SMC_H_LOGZ = 3,
    SMC_H_L = 4,
    SMC_H_ACC0 = 5, /* GMM: accepted proposals of the mean / log-precision / logit blocks */
    SMC_H_ACC1 = 6,
    SMC_H_ACC2 = 7,
    SMC_H_PATH = 8, /* GMM: U_t = sum_i W_i l_i (path-sampling integrand) */
    SMC_H_MON = 9,  /* CV: importance-sampling means of the 4 state rows (cols 9..12) */
    SMC_H_PS = 13,  /* GMM: path-sampling log Z after this step's monitor */
    SMC_HIST_COLS = 16
};

/* Device error word bits (reported by smc_check). */
enum {
    SMC_DEVERR_ZERO_WEIGHTS = 1, /* all weights zero / total not finite at a resample */
    SMC_DEVERR_NONFINITE = 2,    /* NaN log-weight total at a normalisation */
    SMC_DEVERR_GAMMA = 4,        /* gamma sampler exhausted its attempts */
    SMC_DEVERR_TIMEOUT = 8       /* batched step: a wait for other work items timed out */
};

typedef struct smc_config {
    int32_t abi_version; /* SMC_ABI_VERSION */
    int32_t model;       /* smc_model */
    int32_t precision;   /* smc_precision (CV only; GMM is always SMC_F64) */
    int32_t scheme;      /* smc_scheme */
    int64_t n;           /* particles, 1 <= n <= 2^31 - 1 */
    double threshold;    /* resample when ESS < threshold * N; >= 1 always, <= 0 never */
    uint64_t seed;       /* Philox key = (lo32(seed), hi32(seed)) */
    uint32_t problem_id; /* fourth Philox counter word */
    int32_t paper_compatible_loglik; /* CV: drop the Student-t normalising constant */
    /* CV tracking model (Section 5.1.1): standard deviations, time step,
     * Student-t observation noise (obs_nu = +inf selects Gaussian noise). */
    double dt, sd_pos, sd_vel, obs_scale, obs_nu;
    double init_sd[4];
    int32_t n_obs; /* rows of buffers.data ([n_obs][2] observations) */
    /* GMM model (Section 5.2.1): K components, n_data points in buffers.data,
     * priors mu ~ N(mean, sd^2), lambda ~ Gamma(shape, rate), omega ~ Dir(rho). */
    int32_t K;
    int64_t n_data;
    double prior_mu_mean, prior_mu_sd, prior_gamma_shape, prior_gamma_rate, prior_dir_rho;
    int32_t move_kind; /* smc_move_kind */
    int32_t sweeps;    /* default passes over the three blocks per step */
} smc_config;

typedef struct smc_buffers {
    void *state;            /* [rows][n], see the layout above */
    void *state_alt;        /* same size; ping-pong partner (the library swaps them) */
    double *log_weight;     /* [n] */
    int32_t *ancestors;     /* [n] */
    const double *data;     /* CV: observations [n_obs][2]; GMM: y[n_data] */
    double *history;        /* [history_len][SMC_HIST_COLS] or NULL */
    int64_t history_len;
    void *workspace;        /* >= smc_workspace_size() bytes, 256-byte aligned */
    size_t workspace_bytes;
    double *scalars;        /* [SMC_SCALARS_LEN] */
} smc_buffers;

typedef struct smc_move_args {
    int32_t obs_index;     /* CV: observation row that weights this move */
    int32_t fuse_reweight; /* CV: 1 = add the incremental log-weight in the same pass */
    double alpha;          /* GMM: tempering exponent of the MCMC target */
    double scale[3];       /* GMM: per-block random-walk sd or MALA step (mu, eta, z) */
    int32_t sweeps;        /* GMM: passes over the blocks; 0 = config value */
    /* CV with fuse_reweight: when >= 0, the same pass also accumulates the
     * importance-sampling estimate of the INCOMING population (the monitor
     * of step monitor_step, exactly what smc_monitor(ctx, monitor_step, ...)
     * would compute after that step's resample); the following smc_ess
     * completes it into history row monitor_step and, when non-NULL,
     * monitor_out[4] (device).  -1 = off. */
    int32_t monitor_step;
    double *monitor_out;
} smc_move_args;

typedef struct smc_reweight_args {
    int32_t obs_index; /* CV (unfused path): observation row of the increment */
    double dalpha;     /* GMM: alpha_t - alpha_{t-1}; 0 adds exactly 0 */
} smc_reweight_args;

typedef struct smc_ctx smc_ctx;

/* Human-readable name of a status code (static storage). */
const char *smc_status_string(smc_status s);

/* Number of rows of the state arrays and bytes per element for a config. */
smc_status smc_state_rows(const smc_config *cfg, int32_t *rows, int32_t *elem_bytes);

/* Bytes of device workspace the context needs (0 is never returned). */
smc_status smc_workspace_size(const smc_config *cfg, size_t *bytes);

/* Validates the configuration and buffers and binds them to a stream
 * (hipStream_t, NULL = default stream).  Fails with SMC_ERR_DEVICE when no
 * gfx950 device is current.  *out receives the context. */
smc_status smc_create(const smc_config *cfg, const smc_buffers *buf, void *hip_stream,
                      smc_ctx **out);
smc_status smc_destroy(smc_ctx *ctx);
smc_status smc_set_stream(smc_ctx *ctx, void *hip_stream);

/* Initialisation (Algorithm "pf" / Algorithm "gmm", initialisation step):
 * prior draws into the state, initial log-weights (CV: log-likelihood of
 * observation 0; GMM: zero), per-tile weight partials, and the scalar
 * block reset (L = log N, log Z = 0).  Call smc_ess next for the CV model. */
smc_status smc_init(smc_ctx *ctx);

/* Move (Section 4.1 "move" queue, Algorithm "pf" iteration / Algorithm
 * "gmm" MCMC kernel) at counter step `step`.
 *  CV : constant-velocity transition of every particle, reading through the
 *       pending ancestors of the last resample; with fuse_reweight the
 *       incremental log-weight of observation obs_index is added in the
 *       same pass.
 *  GMM: `sweeps` passes of the mean, log-precision and logit Metropolis
 *       blocks (random walk or MALA per config) targeting prior x
 *       likelihood^alpha, reading through pending ancestors. */
smc_status smc_move(smc_ctx *ctx, int32_t step, const smc_move_args *args);

/* Incremental log-weight without moving (Eq. si with the cached
 * likelihood; Eq. inc_weight_mcmc for the GMM: lw += dalpha * l).  CV:
 * weight by observation obs_index at the current state. */
smc_status smc_reweight(smc_ctx *ctx, int32_t step, const smc_reweight_args *args);

/* Normalisation (Section 2.1 ESS; Section 2.2 ratio estimator): combines
 * the per-tile partials of the last move/reweight in fixed order into L,
 * ESS, dlogZ = L - L_prev, log Z, the resampling decision (ESS < tau N) and
 * the cumulative-weight tile offsets; writes history row `step`.  With a
 * non-NULL host pointer it synchronises and returns ESS. */
smc_status smc_ess(smc_ctx *ctx, int32_t step, double *ess_host_or_null);

/* Resampling (Section 2.1) at counter step `step`: when the device decision
 * is 1 (or force != 0) writes sorted ancestors and marks them pending; the
 * next state read applies them and the weights count as equal.  Otherwise
 * does nothing on the device. */
smc_status smc_resample(smc_ctx *ctx, int32_t step, int32_t force);

/* One iteration of Algorithm "pf" (Section 5.1) of a tracking filter: the
 * same as smc_move(step, args), smc_ess(step, NULL) and smc_resample(step,
 * force) in sequence, with the same results bit for bit and the same
 * errors.  The move must carry the weight (args->fuse_reweight = 1; else
 * SMC_ERR_INVALID_ARG, as for a mixture sampler's context, whose iteration
 * takes another order).  For a filter of at most 1024 particles (one tile)
 * with systematic or stratified resampling and no monitor pending from an
 * earlier move, the three are one launch of a single workgroup (a small
 * filter is bound by latency, not by work); otherwise it makes the three
 * calls.  The one-launch form carries no timing events
 * (smc_profile_start). */
smc_status smc_step(smc_ctx *ctx, int32_t step, const smc_move_args *args, int32_t force);

/* Importance-sampling estimate (Section 2.1 estimator 3; Section 4.1
 * monitors) of every state row under the current normalised weights,
 * written to history row `step` (CV: columns SMC_H_MON..; GMM: column
 * SMC_H_PATH gets sum W l) and, when out_dev is non-NULL, to out_dev[rows]
 * (device pointer).
 * GMM: the same call advances the path-sampling estimate of log Z
 * (Section 5.2, path sampling: log Z = integral over alpha of E_alpha[l]) by
 * the trapezoid from the previously monitored step to this one, using the
 * alpha of the last smc_move (0 before any move):
 *   PS += (alpha - alpha_prev) (U + U_prev) / 2,
 * kept in scalars SMC_S_PS_LOGZ and history column SMC_H_PS.  The first
 * monitored step only records (alpha, U); monitoring step 0 (after smc_init
 * and smc_ess) and every step makes the sum run over the whole schedule. */
smc_status smc_monitor(smc_ctx *ctx, int32_t step, double *out_dev);

/* Applies pending ancestors to the state (the value-collection copy of
 * Section 4.1) so that the current state buffer holds the resampled
 * population.  No-op when nothing is pending. */
smc_status smc_gather(smc_ctx *ctx);

/* In-place parent layout of the value-collection copy (Section 4.1,
 * copy(N, copy_from)) for the ancestors of the last resample call:
 * copy_from_dev[j] = j for every particle j with offspring, and the
 * particles without offspring, in ascending order, take the extra copies in
 * ascending (parent, copy) order, so that applying
 * x[j] <- x[copy_from[j]] in place needs no second buffer.  Writes the
 * identity when the last resample call did not resample (device decision).
 * copy_from_dev: device int32[n], caller-owned; enqueued on the context's
 * stream (uses the workspace, so calls on one context must not overlap).
 * Errors: SMC_ERR_INVALID_ARG (null pointer), SMC_ERR_BAD_STATE (before
 * smc_init), SMC_ERR_DEVICE (launch failure). */
smc_status smc_copy_from(smc_ctx *ctx, int32_t *copy_from_dev);

/* Device pointer of the buffer that currently holds the state. */
smc_status smc_current_state(smc_ctx *ctx, void **state);

/* Synchronises the stream and copies the scalar block to host memory. */
smc_status smc_read_scalars(smc_ctx *ctx, double *host_out /* [SMC_SCALARS_LEN] */);

/* Synchronises and maps the device error word: SMC_OK or SMC_ERR_NUMERIC
 * (details in smc_last_error). */
smc_status smc_check(smc_ctx *ctx);
const char *smc_last_error(const smc_ctx *ctx);

/* Mixture log-likelihood and its gradient for n independent parameter
 * vectors (Section 5.2.1 model):
 *   l_i = sum_k log sum_j omega_j N(y_k | mu_j, 1/lambda_j)
 * mu, eta (= log lambda) [K][n], z [K-1][n] (logits against component K),
 * y [n_data]; loglik [n]; grad [3K-1][n] (rows dl/dmu, dl/deta, dl/dz) or
 * NULL.  All device pointers; enqueued on hip_stream. */
smc_status smc_gmm_loglik_grad(const double *mu, const double *eta, const double *z,
                               int64_t n, int32_t K, const double *y, int64_t n_data,
                               double *loglik, double *grad, void *hip_stream);

/* Resampling of caller-held log-weights in one call (Section 2.1: the
 * effective sample size, the resampling decision and the replication
 * numbers R_j with sum N; Eq. resample): normalises lw[n] (unnormalised
 * log-weights) in a fixed order, decides (force != 0: always; else ESS <
 * threshold * n, threshold >= 1 always, <= 0 never) and, when the decision
 * fires, writes the sorted ancestors of `scheme` (SMC_RS_*) drawn from the
 * Philox stream of (seed, step, problem) -- the same ancestors smc_resample
 * writes for a context with these weights -- to ancestors[n]; otherwise
 * leaves ancestors untouched.  summary[5] receives {L = log sum exp lw,
 * L2 = log sum exp 2 lw, ESS, 1 if resampled else 0, device error bits
 * (SMC_DEVERR_*; non-zero means no ancestors were written)}.
 * lw: device double[n], 32-byte aligned, read only; ancestors: device
 * int32[n]; summary: device double[5]; workspace: device memory of at least
 * smc_resample_weights_workspace(n, scheme) bytes, 256-byte aligned, owned
 * by the caller, no initial contents needed, not to be shared by calls that
 * overlap.  Everything is enqueued on hip_stream (the current device's);
 * nothing synchronises.  Errors: SMC_ERR_INVALID_ARG (null or misaligned
 * pointer, n outside [1, 2^31 - 1], unknown scheme, workspace too small),
 * SMC_ERR_DEVICE (no gfx950 device current, launch failure). */
smc_status smc_resample_weights_workspace(int64_t n, int32_t scheme, size_t *bytes);
smc_status smc_resample_weights(const double *lw, int64_t n, int32_t scheme, double threshold,
                                int32_t force, uint64_t seed, uint32_t step, uint32_t problem,
                                int32_t *ancestors, double *summary, void *workspace,
                                size_t workspace_bytes, void *hip_stream);

/* The same resampling for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): arguments, results and errors as smc_resample_weights, but
 * the workspace is the library's own static array of
 * SMC_NOALLOC_SCRATCH_BYTES per device (obtained once per device, held
 * until the process ends); the call allocates nothing.  Every call on a
 * device shares that device's array and leaves its contents behind (the
 * call clears what must start at zero itself), so calls that overlap on
 * one device -- other streams, other threads -- race and must not be
 * issued.  Inputs whose workspace (smc_resample_weights_workspace) exceeds
 * the array are rejected with SMC_ERR_INVALID_ARG: systematic and
 * stratified resampling up to about 100 million particles, multinomial up
 * to about 500 thousand. */
#define SMC_NOALLOC_SCRATCH_BYTES (4u << 20)
smc_status smc_resample_weights_noalloc(const double *lw, int64_t n, int32_t scheme,
                                        double threshold, int32_t force, uint64_t seed,
                                        uint32_t step, uint32_t problem, int32_t *ancestors,
                                        double *summary, void *hip_stream);

/* Raw Philox4x32-10 words of the library's counter-based streams (the
 * per-particle engines of Section 4.1, "Generating random numbers"):
 * out[4*i + w] = word w of the call with counter (i, step, tag<<16 | call,
 * problem) and key (lo32(seed), hi32(seed)), for i = 0..n-1.  out is a
 * device pointer of 4n uint32.  Enqueued on hip_stream. */
smc_status smc_draw_words(uint64_t seed, uint32_t step, uint32_t tag, uint32_t call,
                          uint32_t problem, int64_t n, uint32_t *out, void *hip_stream);

/* Timing of the sweep's dominant kernel by events carried in the kernel's
 * own dispatch, so the stream receives no extra packets: the next `count`
 * launches of the tracking filter's move kernel, or of the mixture
 * sampler's Metropolis kernel (one launch per smc_move: all its blocks and
 * sweeps), of this context are
 * timed (count = 0 disarms).  smc_profile_read waits for them and writes
 * up to `capacity` durations in milliseconds, in launch order; *written
 * receives how many.  The events are timing-only: created without the
 * system-scope fence, so a timed launch ends with the same device-scope
 * release as an untimed one (a system-scope release would add a write-back
 * of the L2 to the measured duration).  Host-side bookkeeping only; events
 * are owned by the context. */
smc_status smc_profile_start(smc_ctx *ctx, int32_t count);
smc_status smc_profile_read(smc_ctx *ctx, float *ms, int32_t capacity, int32_t *written);

/* ------------------------------------------------------------------------
 * Batched form (the paper's two examples, many problems at once): many
 * independent filters and samplers of different sizes advanced together,
 * each step ONE launch of a persistent kernel whose workgroups take work
 * items -- (problem, phase, tile): move / reweight tiles, normalisations,
 * resampling tiles, Metropolis tiles, the samplers' path-sampling monitor
 * (history columns SMC_H_PATH, SMC_H_PS; scalar SMC_S_PS_LOGZ, with the
 * step-0 point taken by smc_batch_init) -- from a queue in ticket order,
 * waiting on per-problem completion counters for the items each depends
 * on.  The queue lists every item after the items it waits for, so the
 * step progresses whatever the number of co-resident workgroups; waits are
 * bounded (a time-out raises SMC_DEVERR_TIMEOUT and the rest of the step is
 * skipped).  A step can be captured once into a HIP graph and replayed.
 * Every problem computes exactly what its own single-problem context would
 * (same per-tile functions, same Philox counters with its problem_id); the
 * batch only changes how the work is scheduled.  Supported: systematic and
 * stratified resampling, FP64 or FP32 tracking state, mixture samplers with
 * up to BATCH_MAX_K = 8 components, any mix of move kinds and sweep counts.
 * ------------------------------------------------------------------------ */
typedef struct smc_batch smc_batch;

typedef struct smc_batch_problem {
    smc_config cfg;          /* as for smc_create (systematic or stratified resampling;
                                mixture samplers with K <= 8) */
    smc_buffers buf;         /* the problem's own device buffers, as for smc_create; the
                                state of step t lives in state (t even) or state_alt
                                (t odd) */
    const double *schedule;  /* mixture samplers: device [schedule_len][4] = alpha_t and
                                the mean, log-precision and logit block scales of step t
                                (row 0: alpha_0 = 0); NULL for tracking filters */
    int32_t schedule_len;    /* mixture samplers: rows of schedule (steps + 1) */
} smc_batch_problem;

/* Device bytes of the batch table (problem descriptors, tile maps, the work
 * queue, completion counters) the caller must provide to smc_batch_create.
 * Validates every configuration (SMC_ERR_INVALID_ARG as smc_create would;
 * SMC_ERR_UNSUPPORTED for multinomial resampling or K > 8). */
smc_status smc_batch_table_size(const smc_batch_problem *probs, int32_t nprob, size_t *bytes);
/* The work queue of one step for these problems, without any device work
 * (for inspection and host-side checks of the schedule): order 0 = the
 * mixture samplers' reweight / normalise / resample items, their Metropolis
 * tiles with the most expensive problems first, then the tracking filters'
 * items; order 1 = phase by phase in problem order.  per_item (1 or 2)
 * 64-particle tiles make one Metropolis item.  items receives *count rows of
 * four int32 {kind (0 move, 1 reweight, 2 normalise, 3 resample, 4
 * Metropolis, 5 monitor), problem, tile, tiles in the item (monitor: the
 * problem's Metropolis items)}; with capacity 0 only
 * *count is written.  SMC_ERR_INVALID_ARG when capacity is non-zero and too
 * small. */
smc_status smc_batch_plan_queue(const smc_batch_problem *probs, int32_t nprob, int32_t order,
                                int32_t per_item, int32_t *items, int64_t capacity,
                                int64_t *count);
/* Builds the batch over caller-owned memory: `table` (device, 256-byte
 * aligned, at least smc_batch_table_size bytes) and every problem's buffers
 * must outlive the batch; all work is enqueued on `hip_stream`, which must
 * not be the legacy null stream when steps are captured.  The step launch
 * starts as many workgroups as the device holds at once (occupancy x
 * compute units) with queue order 0 and one tile per Metropolis item.
 * Errors: SMC_ERR_INVALID_ARG (null or misaligned arguments, a
 * configuration or buffer set smc_create would refuse, a mixture sampler
 * without a schedule, a table that is too small), SMC_ERR_UNSUPPORTED
 * (multinomial resampling, K > 8), SMC_ERR_DEVICE (not a gfx950 device, or
 * a copy failed).  Nothing is created on error. */
smc_status smc_batch_create(const smc_batch_problem *probs, int32_t nprob, void *table,
                            size_t table_bytes, void *hip_stream, smc_batch **out);
/* Releases the host object and its captured graph (not the caller's memory). */
smc_status smc_batch_destroy(smc_batch *b);
/* Autotuner of the step: for every candidate schedule -- queue order (0, 1),
 * 64-particle tiles per Metropolis item (1, 2), step workgroups per compute
 * unit (1 .. the occupancy limit) -- initialises the batch and times
 * `repeats` steps after a warm-up step (median kept), then keeps the
 * fastest.  With a non-NULL cache_path, a line "<arch> <shape buckets> |
 * order=o per_item=q wgs_per_cu=w step_ms=..." (shape buckets: per problem
 * type, mixture size and move kind, the rounded-up log2 of the particle and
 * data counts, with their multiplicities) is read instead of measuring when
 * present, and appended after measuring.  Synchronises the stream.  Leaves
 * the state undefined and drops a captured graph: call smc_batch_init (and
 * capture again) afterwards. */
smc_status smc_batch_autotune(smc_batch *b, int32_t repeats, const char *cache_path);
/* The step's schedule: out[5] = {queue order, tiles per Metropolis item,
 * workgroups per compute unit, workgroups of the launch (workgroups per
 * compute unit times the compute units, at most the items per step), items
 * per step}. */
smc_status smc_batch_schedule(const smc_batch *b, int32_t *out);
/* Sets the step's schedule without measuring: queue order (0, 1), tiles per
 * Metropolis item (1, 2), workgroups per compute unit (clamped to the
 * occupancy limit).  Results do not depend on the schedule, and a run may
 * change it between steps (the steps taken keep their indices).  Copies the
 * new queue to the device (synchronously) and drops a captured graph; not to
 * be called while the stream is being captured. */
smc_status smc_batch_set_schedule(smc_batch *b, int32_t order, int32_t per_item,
                                  int32_t wgs_per_cu);
/* Waves per 64-particle tile of the initialisation of the mixture samplers
 * with K components (SMC_ERR_INVALID_ARG when the batch has none). */
smc_status smc_batch_waves(const smc_batch *b, int32_t K, int32_t *waves);
/* Initialisation of every problem (as smc_init, then the t = 0
 * normalisation and resampling decision); resets the step's queue tickets
 * and completion counters. */
smc_status smc_batch_init(smc_batch *b);
/* Enqueues one step of every problem (the step index follows from the
 * tickets the launch consumes): tracking filters move + weight (completing
 * the previous step's monitor), mixture samplers reweight; all normalise
 * and resample if their ESS is low; mixture samplers then run their
 * Metropolis blocks.  SMC_ERR_BAD_STATE before smc_batch_init or when a
 * problem has no observation / schedule / history row left;
 * SMC_ERR_UNSUPPORTED past the step that the 32-bit ticket and completion
 * counters can index: step t needs t * (work items + workgroups of the
 * step) < 2^32 and t * (tiles of the largest problem: 1024-particle tiles
 * of a filter, 64-particle tiles of a mixture sampler) < 2^32. */
smc_status smc_batch_step(smc_batch *b);
/* Captures one step into a HIP graph (replaces a previous capture); the
 * step index comes from the device, so one capture serves every step. */
smc_status smc_batch_capture(smc_batch *b);
/* Launches the captured step (same checks as smc_batch_step). */
smc_status smc_batch_replay(smc_batch *b);
/* Synchronises and checks every problem's device error word; *first_bad
 * receives the first failing problem or -1 (SMC_ERR_NUMERIC if any). */
smc_status smc_batch_check(smc_batch *b, int32_t *first_bad);
const char *smc_batch_last_error(const smc_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H */
