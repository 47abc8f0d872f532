// smc_core.hip -- model-independent kernels of the SMC sweep on gfx950:
// normalisation (log-sum-exp, ESS, normalising constant, resampling
// decision), resampling to sorted ancestors, importance-sampling monitors
// and the ancestor gather.
#include <math.h>

#include "smc_tiles.hpp"

namespace smc {


// ---------------------------------------------------------------------------
// Scalar block reset (initialisation): L = log N, log Z = 0.
// ---------------------------------------------------------------------------
// Scalars and counters to their t = 0 values; the history rows (whose
// acceptance columns are accumulated) to zero.
__global__ void reset_scalars_kernel(double *scalars, int32_t *counters, int64_t n, double *hist,
                                     int64_t hist_len)
{
    const int t = threadIdx.x;
    if (t < SMC_SCALARS_LEN)
        scalars[t] = 0.0;
    if (t < 16)
        counters[t] = 0;
    if (hist)
        for (int64_t k = t; k < hist_len * SMC_HIST_COLS; k += blockDim.x)
            hist[k] = 0.0;
    __syncthreads();
    if (t == 0) {
        scalars[SMC_S_L] = log((double)n);
        scalars[SMC_S_L2] = log((double)n);
        scalars[SMC_S_ESS] = (double)n;
        scalars[SMC_S_PS_ALPHA] = -1.0;
    }
}

hipError_t launch_reset_scalars(Ctx &c)
{
    hipLaunchKernelGGL(reset_scalars_kernel, dim3(1), dim3(256), 0, c.stream, c.buf.scalars,
                       c.counters(), c.n, c.buf.history, c.buf.history ? c.buf.history_len : 0);
    return hipGetLastError();
}

// Workgroup 0 normalises; workgroup 1 (launched only when monitor partials
// are pending) completes the monitor at the same time.
__global__ __launch_bounds__(FIN_TPB) void finalize_kernel(Prob P, int32_t step, MonDest md)
{
    if (blockIdx.x == 0)
        normalise_block(P, step);
    else
        monitor_block(P, md);
}

// Batched normalisation: two workgroups per problem, the second completing
// (for tracking problems) the monitor of the previous step carried by the
// batched move.
__global__ __launch_bounds__(FIN_TPB) void finalize_batch_kernel(const Prob *__restrict__ probs,
                                                                 const int32_t *__restrict__ step)
{
    const Prob &P = probs[blockIdx.x >> 1];
    const int32_t t = *step;
    if ((blockIdx.x & 1) == 0) {
        normalise_block(P, t);
        return;
    }
    if (P.kind != SMC_MODEL_CV_TRACK || t < 1)
        return;
    MonDest md;
    md.out = nullptr;
    md.scalars = nullptr;
    md.alpha = 0.0;
    md.rows = FIN_MON_ROWS;
    md.hist_col = SMC_H_MON;
    md.hist_ncols = FIN_MON_ROWS;
    md.step = t - 1;
    monitor_block(P, md);
}

hipError_t launch_finalize_batch(const Prob *probs, int32_t nprob, const int32_t *step,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(finalize_batch_kernel, dim3(2 * (unsigned)nprob), dim3(FIN_TPB), 0, s,
                       probs, step);
    return hipGetLastError();
}

__global__ void reset_scalars_batch_kernel(const Prob *__restrict__ probs)
{
    const Prob &P = probs[blockIdx.x];
    const int t = threadIdx.x;
    if (t < SMC_SCALARS_LEN)
        P.scalars[t] = 0.0;
    if (t < 16)
        P.counters[t] = 0;
    if (P.hist)
        for (int64_t k = t; k < P.hist_len * SMC_HIST_COLS; k += blockDim.x)
            P.hist[k] = 0.0;
    __syncthreads();
    if (t == 0) {
        P.scalars[SMC_S_L] = log((double)P.n);
        P.scalars[SMC_S_L2] = log((double)P.n);
        P.scalars[SMC_S_ESS] = (double)P.n;
        P.scalars[SMC_S_PS_ALPHA] = -1.0;
    }
}

__global__ void set_step_kernel(int32_t *step, int32_t value, int32_t add)
{
    if (threadIdx.x == 0)
        *step = add ? *step + value : value;
}

hipError_t launch_reset_scalars_batch(const Prob *probs, int32_t nprob, hipStream_t s)
{
    hipLaunchKernelGGL(reset_scalars_batch_kernel, dim3((unsigned)nprob), dim3(64), 0, s, probs);
    return hipGetLastError();
}

hipError_t launch_set_step(int32_t *step, int32_t value, int32_t add, hipStream_t s)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, s, step, value, add);
    return hipGetLastError();
}

static MonDest mon_dest(const Ctx &c, int32_t step, int rows, double *out)
{
    MonDest d;
    d.step = step;
    d.rows = rows;
    d.out = out;
    d.scalars = nullptr;
    d.alpha = 0.0;
    if (c.cfg.model == SMC_MODEL_CV_TRACK) {
        d.hist_col = SMC_H_MON;
        d.hist_ncols = rows;
    } else {
        d.hist_col = SMC_H_PATH;  // the last monitored row is the log-likelihood
        d.hist_ncols = 1;
        d.scalars = c.buf.scalars;
        d.alpha = c.last_alpha;
    }
    return d;
}

hipError_t launch_finalize(Ctx &c, int32_t step)
{
    MonDest md = mon_dest(c, c.mon_pending_step, c.mon_pending_rows, c.mon_pending_out);
    if (c.mon_pending_step < 0)
        md.step = -1;
    hipLaunchKernelGGL(finalize_kernel, dim3(md.step >= 0 ? 2 : 1), dim3(FIN_TPB), 0, c.stream,
                       make_prob(c), step, md);
    c.mon_pending_step = -1;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One iteration of Algorithm "pf" for a population of one tile (at most 1024
// particles) in a single workgroup: the fused move + weight (Eq. si,
// carrying the monitor of the previous step), the normalisation (Section 2.1
// ESS, Section 2.2 log Z update, then the monitor's completion) and the
// resampling (Section 2.1, Eq. resample).  With one
// workgroup nothing orders the phases but its barriers, so the step's three
// launches become one: each phase reads what the previous one wrote.
// ---------------------------------------------------------------------------
template <typename T, bool MON, bool STRAT>
__global__ __launch_bounds__(TPB) void pf_step_tile_kernel(Prob P, uint32_t t, int32_t obs_index,
                                                           int gather_check, int reset_check,
                                                           MonDest md, int32_t force)
{
    pf_move_tile<T, true, MON>(P, (const T *)P.state[0], (T *)P.state[1], 0, t,
                               P.data + 2 * (int64_t)obs_index, gather_check != 0,
                               reset_check != 0);
    __syncthreads();
    normalise_block<TPB>(P, (int32_t)t);
    if (MON) {
        __syncthreads();
        monitor_block<TPB>(P, md);
    }
    __syncthreads();
    if constexpr (STRAT) {
        __shared__ double sS[TILE];
        __shared__ double sU[RS_UCAP];
        resample_tile<SMC_RS_STRATIFIED>(P, 0, t, force, nullptr, sS, sU);
    } else {
        resample_sys_tile(P, 0, t, force);
    }
}

template <typename T, bool MON>
static void launch_step_tile_t(Ctx &c, const Prob &P, int32_t step, int32_t obs_index,
                               bool gather_check, bool reset_check, const MonDest &md,
                               int32_t force)
{
    if (c.cfg.scheme == SMC_RS_STRATIFIED)
        hipLaunchKernelGGL((pf_step_tile_kernel<T, MON, true>), dim3(1), dim3(TPB), 0, c.stream, P,
                           (uint32_t)step, obs_index, (int)gather_check, (int)reset_check, md,
                           force);
    else
        hipLaunchKernelGGL((pf_step_tile_kernel<T, MON, false>), dim3(1), dim3(TPB), 0, c.stream,
                           P, (uint32_t)step, obs_index, (int)gather_check, (int)reset_check, md,
                           force);
}

hipError_t launch_pf_step_tile(Ctx &c, int32_t step, int32_t obs_index, bool gather_check,
                               bool reset_check, int32_t monitor_step, double *monitor_out,
                               int32_t force)
{
    const Prob P = make_prob(c);
    MonDest md = mon_dest(c, monitor_step, FIN_MON_ROWS, monitor_out);
    const bool mon = monitor_step >= 0;
    if (c.elem_bytes == 4) {
        if (mon)
            launch_step_tile_t<float, true>(c, P, step, obs_index, gather_check, reset_check, md,
                                            force);
        else
            launch_step_tile_t<float, false>(c, P, step, obs_index, gather_check, reset_check, md,
                                             force);
    } else {
        if (mon)
            launch_step_tile_t<double, true>(c, P, step, obs_index, gather_check, reset_check, md,
                                             force);
        else
            launch_step_tile_t<double, false>(c, P, step, obs_index, gather_check, reset_check,
                                              md, force);
    }
    c.cur ^= 1;
    return hipGetLastError();
}

__global__ __launch_bounds__(TPB) void resample_sys_kernel(Prob P, uint32_t t, int32_t force)
{
    resample_sys_tile(P, blockIdx.x, t, force);
}

template <int SCHEME>
__global__ __launch_bounds__(TPB) void resample_merge_kernel(Prob P, uint32_t t, int32_t force,
                                                             const double *__restrict__ G)
{
    __shared__ double sS[TILE];
    __shared__ double sU[RS_UCAP];
    resample_tile<SCHEME>(P, blockIdx.x, t, force, G, sS, sU);
}

// Batched resampling (systematic or stratified) over the tiles of many problems.
__global__ __launch_bounds__(TPB) void resample_batch_kernel(const Prob *__restrict__ probs,
                                                             const int2 *__restrict__ map,
                                                             const int32_t *__restrict__ step)
{
    __shared__ double sS[TILE];
    __shared__ double sU[RS_UCAP];
    const int2 pm = map[blockIdx.x];
    const Prob &P = probs[pm.x];
    if (P.scheme == SMC_RS_STRATIFIED)
        resample_tile<SMC_RS_STRATIFIED>(P, pm.y, (uint32_t)*step, 0, nullptr, sS, sU);
    else
        resample_sys_tile(P, pm.y, (uint32_t)*step, 0);
}

// --- multinomial: cumulative sums G of N+1 exponentials -------------------

__device__ __forceinline__ double mn_exp(Key key, int64_t k, uint32_t t, uint32_t p)
{
    const uint4 w = draw(key, (uint32_t)k, t, TAG_RESAMPLE, 1, p);
    return -log(u53(w.x, w.y));
}

__global__ __launch_bounds__(TPB) void mn_tile_sum_kernel(const double *__restrict__ scalars,
                                                          int32_t force, int64_t count, Key key,
                                                          uint32_t t, uint32_t p,
                                                          double *__restrict__ gtile)
{
    __shared__ double red[NWAVES];
    if (!(force != 0 || scalars[SMC_S_FLAG] != 0.0))
        return;
    const int64_t base = (int64_t)blockIdx.x * TILE;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        if (i < count)
            s += mn_exp(key, i, t, p);
    }
    s = block_sum<NWAVES>(s, red);
    if (threadIdx.x == 0)
        gtile[blockIdx.x] = s;
}

__global__ __launch_bounds__(FIN_TPB) void mn_prefix_kernel(const double *__restrict__ scalars,
                                                            int32_t force,
                                                            const double *__restrict__ gtile,
                                                            int64_t gtiles,
                                                            double *__restrict__ gprefix)
{
    __shared__ double red[FIN_NW];
    if (!(force != 0 || scalars[SMC_S_FLAG] != 0.0))
        return;
    tile_offsets(gtiles, [&](int64_t b) { return gtile[b]; }, gprefix, red);
}

__global__ __launch_bounds__(TPB) void mn_write_kernel(const double *__restrict__ scalars,
                                                       int32_t force, int64_t count, Key key,
                                                       uint32_t t, uint32_t p,
                                                       const double *__restrict__ gprefix,
                                                       double *__restrict__ G)
{
    __shared__ double red[NWAVES];
    if (!(force != 0 || scalars[SMC_S_FLAG] != 0.0))
        return;
    const int64_t b = blockIdx.x;
    const int64_t base = b * TILE;
    const int len = (int)min((int64_t)TILE, count - base);
    const double P0 = gprefix[b], P1 = gprefix[b + 1];
    double carry = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        const double e = i < count ? mn_exp(key, i, t, p) : 0.0;
        double tot;
        const double incl = block_incl_scan<NWAVES>(e, red, &tot);
        if (i < count)
            G[i] = (k * TPB + (int)threadIdx.x == len - 1) ? P1 : fmin(P0 + (carry + incl), P1);
        carry += tot;
    }
}

hipError_t launch_resample(Ctx &c, int32_t step, int32_t force)
{
    const Prob P = make_prob(c);
    const Key key = make_key(c.cfg.seed);
    const uint32_t p = c.cfg.problem_id;
    const dim3 grid((unsigned)c.ntiles);
    switch (c.cfg.scheme) {
    case SMC_RS_SYSTEMATIC:
        hipLaunchKernelGGL(resample_sys_kernel, grid, dim3(TPB), 0, c.stream, P, (uint32_t)step,
                           force);
        break;
    case SMC_RS_STRATIFIED:
        hipLaunchKernelGGL(resample_merge_kernel<SMC_RS_STRATIFIED>, grid, dim3(TPB), 0, c.stream,
                           P, (uint32_t)step, force, (const double *)nullptr);
        break;
    default: {
        const int64_t count = c.n + 1;
        hipLaunchKernelGGL(mn_tile_sum_kernel, dim3((unsigned)c.gtiles), dim3(TPB), 0, c.stream,
                           c.buf.scalars, force, count, key, (uint32_t)step, p, c.gtile());
        hipLaunchKernelGGL(mn_prefix_kernel, dim3(1), dim3(FIN_TPB), 0, c.stream, c.buf.scalars,
                           force, c.gtile(), c.gtiles, c.gprefix());
        hipLaunchKernelGGL(mn_write_kernel, dim3((unsigned)c.gtiles), dim3(TPB), 0, c.stream,
                           c.buf.scalars, force, count, key, (uint32_t)step, p, c.gprefix(),
                           c.g());
        hipLaunchKernelGGL(resample_merge_kernel<SMC_RS_MULTINOMIAL>, grid, dim3(TPB), 0,
                           c.stream, P, (uint32_t)step, force, (const double *)c.g());
    }
    }
    return hipGetLastError();
}

hipError_t launch_resample_batch(const Prob *probs, const int2 *map, int64_t tiles,
                                 const int32_t *step, hipStream_t s)
{
    if (tiles == 0)
        return hipSuccess;
    hipLaunchKernelGGL(resample_batch_kernel, dim3((unsigned)tiles), dim3(TPB), 0, s, probs, map,
                       step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Resampling of a caller's log-weights in one call: per-tile partials of
// lw, the normalisation, the resampling of the configured scheme, and a
// five-value summary.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void lw_partials_kernel(const double *__restrict__ lw,
                                                          int64_t n,
                                                          TilePartial *__restrict__ part)
{
    __shared__ double red[NWAVES];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    double l[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        l[k] = i < n ? lw[i] : -INFINITY;
    }
    tile_partial(l, part + blockIdx.x, red);
}

// summary = {L, L2, ESS, resampled (0/1), device error bits}
__global__ void resample_summary_kernel(const double *__restrict__ scalars,
                                        const int32_t *__restrict__ counters,
                                        double *__restrict__ summary)
{
    if (threadIdx.x == 0) {
        summary[0] = scalars[SMC_S_RESAMPLED] != 0.0 ? scalars[SMC_S_LPRE] : scalars[SMC_S_L];
        summary[1] = scalars[SMC_S_L2];
        summary[2] = scalars[SMC_S_ESS];
        summary[3] = scalars[SMC_S_RESAMPLED];
        summary[4] = (double)counters[CNT_ERR];
    }
}

hipError_t launch_resample_weights(Ctx &c, int32_t step, int32_t force, double *summary)
{
    hipError_t e = launch_reset_scalars(c);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(lw_partials_kernel, dim3((unsigned)c.ntiles), dim3(TPB), 0, c.stream,
                       (const double *)c.buf.log_weight, c.n, c.partials());
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    c.mon_pending_step = -1;
    if ((e = launch_finalize(c, -1)) != hipSuccess)
        return e;
    if ((e = launch_resample(c, step, force)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(resample_summary_kernel, dim3(1), dim3(64), 0, c.stream, c.buf.scalars,
                       (const int32_t *)c.counters(), summary);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Monitors: per-tile sums of w_i and w_i x_r,i (w_i = exp(lw_i - M), or 1
// after a resample), column-major [1 + rows][ntiles], then one workgroup
// combines the tiles in a fixed order.
// ---------------------------------------------------------------------------
constexpr int MON_GROUP = 8;

template <typename T>
__global__ __launch_bounds__(TPB) void mon_partial_kernel(
    const T *__restrict__ x, int rows, int64_t n, const double *__restrict__ lw,
    const int32_t *__restrict__ anc, const double *__restrict__ scalars, int gather_check,
    int reset_check, double *__restrict__ mon, int64_t ntiles)
{
    __shared__ double red[NWAVES * MON_GROUP];
    const bool resampled = scalars[SMC_S_RESAMPLED] != 0.0;
    const bool gather = gather_check && resampled;
    const bool reset = reset_check && resampled;
    const double M = scalars[SMC_S_M];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    double w[ITEMS];
    int64_t src[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        w[k] = 0.0;
        src[k] = 0;
        if (i < n) {
            src[k] = gather ? (int64_t)anc[i] : i;
            w[k] = reset ? 1.0 : exp_nonpos_d(lw[i] - M);
        }
    }
    // column 0 = sum w, column 1 + r = sum w x_r; eight columns per barrier pair
    for (int c0 = 0; c0 <= rows; c0 += MON_GROUP) {
        double s[MON_GROUP];
#pragma unroll
        for (int g = 0; g < MON_GROUP; ++g) {
            const int c = c0 + g;
            s[g] = 0.0;
            if (c == 0) {
                s[g] = ((w[0] + w[1]) + w[2]) + w[3];
            } else if (c <= rows) {
#pragma unroll
                for (int k = 0; k < ITEMS; ++k)
                    if (w[k] != 0.0)
                        s[g] += w[k] * (double)x[(int64_t)(c - 1) * n + src[k]];
            }
        }
        block_sum_n<NWAVES, MON_GROUP>(s, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int g = 0; g < MON_GROUP; ++g)
                if (c0 + g <= rows)
                    mon[(int64_t)(c0 + g) * ntiles + blockIdx.x] = s[g];
        }
    }
}

// The same partials per 64-particle tile: one wave per workgroup, one
// particle per lane, no barriers.  Many more workgroups for the same work,
// which is what a population too small to fill the chip with 1024-particle
// tiles needs.
template <typename T>
__global__ __launch_bounds__(WAVE) void mon_partial64_kernel(
    const T *__restrict__ x, int rows, int64_t n, const double *__restrict__ lw,
    const int32_t *__restrict__ anc, const double *__restrict__ scalars, int gather_check,
    int reset_check, double *__restrict__ mon, int64_t ntiles)
{
    const bool resampled = scalars[SMC_S_RESAMPLED] != 0.0;
    const bool gather = gather_check && resampled;
    const bool reset = reset_check && resampled;
    const double M = scalars[SMC_S_M];
    const int64_t i = (int64_t)blockIdx.x * WAVE + lane_id();
    double w = 0.0;
    int64_t src = 0;
    if (i < n) {
        src = gather ? (int64_t)anc[i] : i;
        w = reset ? 1.0 : exp_nonpos_d(lw[i] - M);
    }
    for (int c0 = 0; c0 <= rows; c0 += MON_GROUP) {
        double v[MON_GROUP];
#pragma unroll
        for (int g = 0; g < MON_GROUP; ++g) {
            const int c = c0 + g;
            v[g] = 0.0;
            if (c == 0)
                v[g] = w;
            else if (c <= rows && w != 0.0)
                v[g] = w * (double)x[(int64_t)(c - 1) * n + src];
        }
#pragma unroll
        for (int g = 0; g < MON_GROUP; ++g)
            v[g] = wave_sum(v[g]);
        if (lane_id() == 0) {
#pragma unroll
            for (int g = 0; g < MON_GROUP; ++g)
                if (c0 + g <= rows)
                    mon[(int64_t)(c0 + g) * ntiles + blockIdx.x] = v[g];
        }
    }
}

__global__ __launch_bounds__(FIN_TPB) void mon_final_kernel(const double *__restrict__ mon,
                                                            int64_t ntiles, MonDest md,
                                                            double *__restrict__ hist,
                                                            int64_t hist_len)
{
    __shared__ double red[MON_STRIDE * FIN_NW];
    __shared__ double col[MON_STRIDE];
    mon_combine<FIN_TPB>(mon, ntiles, md, hist, hist_len, red, col);
}

hipError_t launch_monitor(Ctx &c, int32_t step, double *out_dev, int rows, bool gather_pending,
                          bool reset_pending)
{
    // 64-particle tiles up to MON64_MAX_TILES of them, 1024-particle tiles beyond
    const int64_t t64 = ceil_div(c.n, WAVE);
    const bool small = t64 <= MON64_MAX_TILES;
    const int64_t ntm = small ? t64 : c.ntiles;
    const dim3 grid((unsigned)ntm);
#define SMC_MON_ARGS(T)                                                                          \
    (const T *)c.state_ptr(), rows, c.n, c.buf.log_weight, c.buf.ancestors, c.buf.scalars,       \
        (int)gather_pending, (int)reset_pending, c.mon(), ntm
    if (small && c.elem_bytes == 4)
        hipLaunchKernelGGL(mon_partial64_kernel<float>, grid, dim3(WAVE), 0, c.stream,
                           SMC_MON_ARGS(float));
    else if (small)
        hipLaunchKernelGGL(mon_partial64_kernel<double>, grid, dim3(WAVE), 0, c.stream,
                           SMC_MON_ARGS(double));
    else if (c.elem_bytes == 4)
        hipLaunchKernelGGL(mon_partial_kernel<float>, grid, dim3(TPB), 0, c.stream,
                           SMC_MON_ARGS(float));
    else
        hipLaunchKernelGGL(mon_partial_kernel<double>, grid, dim3(TPB), 0, c.stream,
                           SMC_MON_ARGS(double));
#undef SMC_MON_ARGS
    const MonDest md = mon_dest(c, step, rows, out_dev);
    hipLaunchKernelGGL(mon_final_kernel, dim3(1), dim3(FIN_TPB), 0, c.stream, c.mon(), ntm, md,
                       c.buf.history, c.buf.history_len);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Standalone gather (value-collection copy): out[r][i] = in[r][a_i] when a
// resample is pending, else a plain copy.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(TPB) void gather_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                     int rows, int64_t n,
                                                     const int32_t *__restrict__ anc,
                                                     const double *__restrict__ scalars)
{
    const bool gather = scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= n)
        return;
    const int64_t src = gather ? (int64_t)anc[i] : i;
    for (int r = 0; r < rows; ++r)
        out[(int64_t)r * n + i] = in[(int64_t)r * n + src];
}

hipError_t launch_gather(Ctx &c)
{
    const dim3 grid((unsigned)ceil_div(c.n, TPB));
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(gather_kernel<float>, grid, dim3(TPB), 0, c.stream,
                           (const float *)c.state_ptr(), (float *)c.other_ptr(), c.state_rows,
                           c.n, c.buf.ancestors, c.buf.scalars);
    else
        hipLaunchKernelGGL(gather_kernel<double>, grid, dim3(TPB), 0, c.stream,
                           (const double *)c.state_ptr(), (double *)c.other_ptr(), c.state_rows,
                           c.n, c.buf.ancestors, c.buf.scalars);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// In-place parent layout of the value-collection copy (Section 4.1,
// copy(N, copy_from)): every particle with offspring keeps its own index,
// copy_from[j] = j, and the indices of the particles without offspring, in
// ascending order, receive the extra copies in ascending (parent, copy)
// order.  With the sorted ancestors a those extra copies are exactly the
// slots i > 0 with a_i == a_{i-1}, in slot order.  So: mark the particles
// that appear (at the first slot of each run of equal ancestors), rank the
// duplicate slots and the empty particles by exclusive scans over tiles,
// scatter each duplicate's parent to its rank, and let every empty particle
// take the parent of the same rank.  Without a resample (device flag 0) the
// layout is the identity.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void cf_clear_kernel(const double *__restrict__ scalars,
                                                       int32_t *__restrict__ present, int64_t n)
{
    if (scalars[SMC_S_RESAMPLED] == 0.0)
        return;
    const int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < n)
        present[i] = 0;
}

// Slot tile b: marks the parents of the run starts, counts the duplicates.
__global__ __launch_bounds__(TPB) void cf_mark_kernel(const double *__restrict__ scalars,
                                                      const int32_t *__restrict__ anc, int64_t n,
                                                      int32_t *__restrict__ present,
                                                      double *__restrict__ cnt_dup)
{
    __shared__ double red[NWAVES];
    if (scalars[SMC_S_RESAMPLED] == 0.0)
        return;
    const int64_t base = (int64_t)blockIdx.x * TILE + ITEMS * threadIdx.x;
    double dups = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            const int32_t a = anc[i];
            if (i == 0 || anc[i - 1] != a)
                present[a] = 1;
            else
                dups += 1.0;
        }
    }
    dups = block_sum<NWAVES>(dups, red);
    if (threadIdx.x == 0)
        cnt_dup[blockIdx.x] = dups;
}

// Particle tile b: counts the particles without offspring.
__global__ __launch_bounds__(TPB) void cf_count_empty_kernel(const double *__restrict__ scalars,
                                                             const int32_t *__restrict__ present,
                                                             int64_t n,
                                                             double *__restrict__ cnt_empty)
{
    __shared__ double red[NWAVES];
    if (scalars[SMC_S_RESAMPLED] == 0.0)
        return;
    const int64_t base = (int64_t)blockIdx.x * TILE + ITEMS * threadIdx.x;
    double e = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (base + k < n && present[base + k] == 0)
            e += 1.0;
    e = block_sum<NWAVES>(e, red);
    if (threadIdx.x == 0)
        cnt_empty[blockIdx.x] = e;
}

// One workgroup: exclusive tile offsets of both counts (integer-valued, so
// exact in double precision).
__global__ __launch_bounds__(FIN_TPB) void cf_scan_kernel(const double *__restrict__ scalars,
                                                          const double *__restrict__ cnt_dup,
                                                          const double *__restrict__ cnt_empty,
                                                          int64_t ntiles,
                                                          double *__restrict__ off_dup,
                                                          double *__restrict__ off_empty)
{
    __shared__ double red[2 * FIN_NW];
    if (scalars[SMC_S_RESAMPLED] == 0.0)
        return;
    tile_offsets(ntiles, [&](int64_t b) { return cnt_dup[b]; }, off_dup, red);
    __syncthreads();
    tile_offsets(ntiles, [&](int64_t b) { return cnt_empty[b]; }, off_empty, red);
}

// Slot tile b: each duplicate slot writes its parent at its rank.
__global__ __launch_bounds__(TPB) void cf_dup_kernel(const double *__restrict__ scalars,
                                                     const int32_t *__restrict__ anc, int64_t n,
                                                     const double *__restrict__ off_dup,
                                                     int32_t *__restrict__ dup_parent)
{
    __shared__ double red[NWAVES];
    if (scalars[SMC_S_RESAMPLED] == 0.0)
        return;
    const int64_t base = (int64_t)blockIdx.x * TILE + ITEMS * threadIdx.x;
    int32_t a[ITEMS];
    bool dup[ITEMS];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k;
        a[k] = i < n ? anc[i] : 0;
        dup[k] = i < n && i > 0 && anc[i - 1] == a[k];
        run += dup[k] ? 1.0 : 0.0;
    }
    double total;
    double r = block_excl_scan<NWAVES>(run, red, &total) + off_dup[blockIdx.x];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        if (dup[k]) {
            dup_parent[(int64_t)r] = a[k];
            r += 1.0;
        }
}

// Particle tile b: the layout itself.
__global__ __launch_bounds__(TPB) void cf_final_kernel(const double *__restrict__ scalars,
                                                       const int32_t *__restrict__ present,
                                                       int64_t n,
                                                       const double *__restrict__ off_empty,
                                                       const int32_t *__restrict__ dup_parent,
                                                       int32_t *__restrict__ out)
{
    __shared__ double red[NWAVES];
    const bool resampled = scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t base = (int64_t)blockIdx.x * TILE + ITEMS * threadIdx.x;
    if (!resampled) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (base + k < n)
                out[base + k] = (int32_t)(base + k);
        return;
    }
    bool empty[ITEMS];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        empty[k] = base + k < n && present[base + k] == 0;
        run += empty[k] ? 1.0 : 0.0;
    }
    double total;
    double r = block_excl_scan<NWAVES>(run, red, &total) + off_empty[blockIdx.x];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t j = base + k;
        if (j < n) {
            if (empty[k]) {
                out[j] = dup_parent[(int64_t)r];
                r += 1.0;
            } else {
                out[j] = (int32_t)j;
            }
        }
    }
}

hipError_t launch_copy_from(Ctx &c, int32_t *out)
{
    const int64_t n = c.n, nt = c.ntiles;
    const double *sc = c.buf.scalars;
    int32_t *present = c.cf_present();
    int32_t *dup_parent = c.cf_dup();
    double *cnt_dup = c.cf_tiles(), *cnt_empty = cnt_dup + nt;
    double *off_dup = cnt_empty + nt, *off_empty = off_dup + (nt + 1);
    hipLaunchKernelGGL(cf_clear_kernel, dim3((unsigned)ceil_div(n, TPB)), dim3(TPB), 0, c.stream,
                       sc, present, n);
    hipLaunchKernelGGL(cf_mark_kernel, dim3((unsigned)nt), dim3(TPB), 0, c.stream, sc,
                       (const int32_t *)c.buf.ancestors, n, present, cnt_dup);
    hipLaunchKernelGGL(cf_count_empty_kernel, dim3((unsigned)nt), dim3(TPB), 0, c.stream, sc,
                       (const int32_t *)present, n, cnt_empty);
    hipLaunchKernelGGL(cf_scan_kernel, dim3(1), dim3(FIN_TPB), 0, c.stream, sc,
                       (const double *)cnt_dup, (const double *)cnt_empty, nt, off_dup, off_empty);
    hipLaunchKernelGGL(cf_dup_kernel, dim3((unsigned)nt), dim3(TPB), 0, c.stream, sc,
                       (const int32_t *)c.buf.ancestors, n, (const double *)off_dup, dup_parent);
    hipLaunchKernelGGL(cf_final_kernel, dim3((unsigned)nt), dim3(TPB), 0, c.stream, sc,
                       (const int32_t *)present, n, (const double *)off_empty,
                       (const int32_t *)dup_parent, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Raw words of the counter-based streams (for external checks and users).
// ---------------------------------------------------------------------------
__global__ void draw_words_kernel(Key key, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                                  int64_t n, uint4 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = draw(key, (uint32_t)i, t, tag, j, p);
}

hipError_t launch_draw_words(uint64_t seed, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                             int64_t n, uint32_t *out, hipStream_t stream)
{
    hipLaunchKernelGGL(draw_words_kernel, dim3((unsigned)ceil_div(n, TPB)), dim3(TPB), 0, stream,
                       make_key(seed), t, tag, j, p, n, reinterpret_cast<uint4 *>(out));
    return hipGetLastError();
}

}  // namespace smc
