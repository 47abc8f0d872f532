// smc_core.hip -- model-independent kernels of the SMC sweep on gfx950:
// normalisation (log-sum-exp, ESS, normalising constant, resampling
// decision), resampling to sorted ancestors, importance-sampling monitors
// and the ancestor gather.
#include <math.h>

#include "smc_internal.hpp"

namespace smc {


// ---------------------------------------------------------------------------
// Scalar block reset (initialisation): L = log N, log Z = 0.
// ---------------------------------------------------------------------------
__global__ void reset_scalars_kernel(double *scalars, int32_t *counters, int64_t n)
{
    const int t = threadIdx.x;
    if (t < SMC_SCALARS_LEN)
        scalars[t] = 0.0;
    if (t < 16)
        counters[t] = 0;
    __syncthreads();
    if (t == 0) {
        scalars[SMC_S_L] = log((double)n);
        scalars[SMC_S_L2] = log((double)n);
        scalars[SMC_S_ESS] = (double)n;
    }
}

hipError_t launch_reset_scalars(Ctx &c)
{
    hipLaunchKernelGGL(reset_scalars_kernel, dim3(1), dim3(64), 0, c.stream, c.buf.scalars,
                       c.counters(), c.n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cumulative offsets of `count` non-negative tile values v_b (computed by
// `val(b)`) in one workgroup of FIN_PASS_TPB lanes: out[b] = sum_{b' < b} v_b',
// out[count] = total.  Values are staged through LDS in passes of FIN_PASS;
// each lane sums a contiguous chunk of FIN_CH values sequentially, the
// chunk totals are scanned across the workgroup in a fixed order, and an
// exact running maximum keeps out[] non-decreasing.  The same inputs always
// give the same outputs.
// ---------------------------------------------------------------------------
constexpr int FIN_CH = 16;
constexpr int FIN_PASS_TPB = 256;
constexpr int FIN_PASS = FIN_PASS_TPB * FIN_CH;
constexpr int FIN_LDS = FIN_PASS_TPB * (FIN_CH + 1);  // padded chunks: no bank conflicts

__device__ __forceinline__ int fin_pidx(int j) { return (j / FIN_CH) * (FIN_CH + 1) + j % FIN_CH; }

template <typename F>
__device__ double tile_offsets(int64_t count, F val, double *out, double *sv, double *red)
{
    constexpr int NW = FIN_PASS_TPB / WAVE;
    const int tid = threadIdx.x;
    double carry = 0.0;
    for (int64_t pbase = 0; pbase < count; pbase += FIN_PASS) {
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < FIN_CH; ++k) {
            const int j = k * FIN_PASS_TPB + tid;
            const int64_t b = pbase + j;
            sv[fin_pidx(j)] = b < count ? val(b) : 0.0;
        }
        __syncthreads();
        double e[FIN_CH];
        double run = 0.0;
#pragma unroll
        for (int j = 0; j < FIN_CH; ++j) {
            e[j] = run;
            run += sv[tid * (FIN_CH + 1) + j];
        }
        double total;
        const double excl = block_excl_scan<NW>(run, red, &total);
        // candidate offsets, then the exact floor from all earlier chunks
        double last = 0.0;
#pragma unroll
        for (int j = 0; j < FIN_CH; ++j) {
            e[j] = carry + (excl + e[j]);
            last = fmax(last, e[j]);
        }
        const double incl_max = block_incl_max_scan<NW>(last, red);
        double floor_v = __shfl_up(incl_max, 1);
        __syncthreads();
        if (lane_id() == WAVE - 1)
            red[wave_id()] = incl_max;
        __syncthreads();
        if (lane_id() == 0)
            floor_v = wave_id() == 0 ? carry : red[wave_id() - 1];
        floor_v = fmax(floor_v, carry);
#pragma unroll
        for (int j = 0; j < FIN_CH; ++j) {
            const int64_t b = pbase + (int64_t)tid * FIN_CH + j;
            if (b < count)
                out[b] = fmax(e[j], floor_v);
        }
        const double pass_max = red[NW - 1];
        carry = fmax(carry + total, pass_max);
    }
    if (tid == 0)
        out[count] = carry;
    return carry;
}

// ---------------------------------------------------------------------------
// Normalisation (single workgroup): global max M, tile offsets of the
// cumulative weights, S1 = sum exp(lw - M), S2 = sum exp(2 (lw - M)),
// L = M + log S1, L2 = 2M + log S2, ESS = exp(2L - L2), dlogZ = L - L_prev,
// decision ESS < tau N (tau >= 1 always, tau <= 0 never).  When a move
// carried the monitor partials of the previous step (mon_step >= 0), their
// importance-sampling estimates are completed here as well.
// ---------------------------------------------------------------------------
struct MonDest {
    int32_t step;     // history row, or -1 when no monitor partials are pending
    int rows;         // monitored rows (partial columns 1..rows; column 0 = sum w)
    int hist_col;     // first history column receiving estimates
    int hist_ncols;   // how many of the last rows go to the history
    double *out;      // optional device output [rows]
};

__device__ void mon_combine(const double *__restrict__ mon, int64_t ntiles, const MonDest &d,
                            double *__restrict__ hist, int64_t hist_len, double *red,
                            double *col)
{
    constexpr int NW = FIN_PASS_TPB / WAVE;
    for (int r = 0; r <= d.rows; ++r) {
        double a = 0.0;
        for (int64_t b = threadIdx.x; b < ntiles; b += FIN_PASS_TPB)
            a += mon[(int64_t)r * ntiles + b];
        a = block_sum<NW>(a, red);
        if (threadIdx.x == 0)
            col[r] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < d.rows) {
        const int r = threadIdx.x;
        const double est = col[1 + r] / col[0];
        if (d.out)
            d.out[r] = est;
        if (hist && d.step >= 0 && d.step < hist_len && r >= d.rows - d.hist_ncols)
            hist[(int64_t)d.step * SMC_HIST_COLS + d.hist_col + (r - (d.rows - d.hist_ncols))] =
                est;
    }
}

__global__ __launch_bounds__(FIN_PASS_TPB) void finalize_kernel(
    const TilePartial *__restrict__ part, int64_t ntiles, int64_t n, double threshold,
    double *__restrict__ prefix, double *__restrict__ scalars, double *__restrict__ hist,
    int64_t hist_len, int32_t step, int32_t *__restrict__ counters,
    const double *__restrict__ mon, MonDest md)
{
    constexpr int NW = FIN_PASS_TPB / WAVE;
    __shared__ double sv[FIN_LDS];
    __shared__ double red[NW];
    __shared__ double col[MON_STRIDE];
    const int tid = threadIdx.x;
    double m = -INFINITY;
    for (int64_t b = tid; b < ntiles; b += FIN_PASS_TPB)
        m = fmax(m, part[b].m);
    const double M = block_max<NW>(m, red);
    auto scale = [&](int64_t b) {
        const double mb = part[b].m;
        return mb > -INFINITY ? exp(mb - M) : 0.0;
    };
    const double S1 = tile_offsets(
        ntiles, [&](int64_t b) { return part[b].s1 * scale(b); }, prefix, sv, red);
    double s2 = 0.0;
    for (int64_t b = tid; b < ntiles; b += FIN_PASS_TPB) {
        const double sc = scale(b);
        s2 += part[b].s2 * (sc * sc);
    }
    const double S2 = block_sum<NW>(s2, red);
    if (md.step >= 0)
        mon_combine(mon, ntiles, md, hist, hist_len, red, col);
    if (tid == 0) {
        const double L = M + log(S1);
        const double L2 = 2.0 * M + log(S2);
        const double ess = exp(2.0 * L - L2);
        const double Lprev = scalars[SMC_S_L];
        const double dlogz = L - Lprev;
        const double logz = scalars[SMC_S_LOGZ] + dlogz;
        int flag;
        if (threshold >= 1.0)
            flag = 1;
        else if (threshold <= 0.0)
            flag = 0;
        else
            flag = ess < threshold * (double)n;
        if (!(S1 > 0.0) || !isfinite(S1) || !isfinite(M)) {
            atomicOr(&counters[CNT_ERR], SMC_DEVERR_NONFINITE);
            flag = 0;
        }
        scalars[SMC_S_L] = L;
        scalars[SMC_S_L2] = L2;
        scalars[SMC_S_ESS] = ess;
        scalars[SMC_S_DLOGZ] = dlogz;
        scalars[SMC_S_LOGZ] = logz;
        scalars[SMC_S_FLAG] = (double)flag;
        scalars[SMC_S_M] = M;
        scalars[SMC_S_STOT] = S1;
        if (hist && step >= 0 && step < hist_len) {
            double *h = hist + (int64_t)step * SMC_HIST_COLS;
            h[SMC_H_ESS] = ess;
            h[SMC_H_FLAG] = (double)flag;
            h[SMC_H_DLOGZ] = dlogz;
            h[SMC_H_LOGZ] = logz;
            h[SMC_H_L] = L;
        }
    }
}

static MonDest mon_dest(const Ctx &c, int32_t step, int rows, double *out)
{
    MonDest d;
    d.step = step;
    d.rows = rows;
    d.out = out;
    if (c.cfg.model == SMC_MODEL_CV_TRACK) {
        d.hist_col = SMC_H_MON;
        d.hist_ncols = rows;
    } else {
        d.hist_col = SMC_H_PATH;  // the last monitored row is the log-likelihood
        d.hist_ncols = 1;
    }
    return d;
}

hipError_t launch_finalize(Ctx &c, int32_t step)
{
    MonDest md = mon_dest(c, c.mon_pending_step, c.mon_pending_rows, c.mon_pending_out);
    if (c.mon_pending_step < 0)
        md.step = -1;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_PASS_TPB), 0, c.stream, c.partials(),
                       c.ntiles, c.n, c.cfg.threshold, c.prefix(), c.buf.scalars, c.buf.history,
                       c.buf.history_len, step, c.counters(), c.mon(), md);
    c.mon_pending_step = -1;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Resampling.  Ordered uniforms u_i and the cumulative weights S_j (tile
// offsets from the normalisation plus a workgroup scan inside each tile,
// clamped to stay monotone and to end exactly on the next tile's offset)
// give a_i = min{ j : S_j > u_i S }.  Each tile owns the contiguous slot
// range [c(S_start), c(S_end)) where c(x) = #{ i : u_i S < x }, and fills it
// with a binary search of its own S values held in LDS.
// ---------------------------------------------------------------------------

struct SysPred {  // u_i = (i + U) / N
    double U, stot;
    int64_t n;
    __device__ double operator()(int64_t i) const
    {
        return (((double)i + U) / (double)n) * stot;
    }
};

struct StratPred {  // u_i = (i + U_i) / N, U_i from counter (i, t, RESAMPLE, 0)
    Key key;
    uint32_t t, p;
    double stot;
    int64_t n;
    __device__ double operator()(int64_t i) const
    {
        const uint4 w = draw(key, (uint32_t)i, t, TAG_RESAMPLE, 0, p);
        return (((double)i + u53(w.x, w.y)) / (double)n) * stot;
    }
};

struct MultiPred {  // u_i = G_i / G_N
    const double *G;
    double gn, stot;
    int64_t n;
    __device__ double operator()(int64_t i) const { return (G[i] / gn) * stot; }
};

// Smallest i in [0, n] with pred(i) >= x (n when none), starting from an
// estimate that is exact up to rounding and walking to the exact answer.
template <typename P>
__device__ int64_t count_below_walk(const P &pred, double x, int64_t n, double est)
{
    int64_t i;
    if (!(est > 0.0))
        i = 0;
    else if (est >= (double)n)
        i = n;
    else
        i = (int64_t)est;
    while (i > 0 && pred(i - 1) >= x)
        --i;
    while (i < n && pred(i) < x)
        ++i;
    return i;
}

// Same answer by a 64-way search of one wave (pred monotone; pred(n) = +inf).
template <typename P>
__device__ int64_t count_below_search(const P &pred, double x, int64_t n)
{
    const int lane = lane_id();
    int64_t lo = 0, hi = n;
    while (hi - lo > WAVE) {
        const int64_t span = hi - lo;
        const int64_t pos = lo + (span * lane) / WAVE;
        const bool q = pred(pos) >= x;
        const unsigned long long bal = __ballot(q);
        if (bal == 0ull) {
            lo = lo + (span * (WAVE - 1)) / WAVE + 1;
        } else {
            const int f = __ffsll((long long)bal) - 1;
            if (f == 0) {
                hi = lo;
                break;
            }
            hi = lo + (span * f) / WAVE;
            lo = lo + (span * (f - 1)) / WAVE + 1;
        }
    }
    const int64_t pos = lo + lane;
    const bool q = pos < hi ? pred(pos) >= x : false;
    const unsigned long long bal = __ballot(q);
    if (bal == 0ull)
        return hi;
    return lo + (__ffsll((long long)bal) - 1);
}

template <int SCHEME>
__global__ __launch_bounds__(TPB) void resample_kernel(
    const double *__restrict__ lw, const TilePartial *__restrict__ part,
    const double *__restrict__ prefix, int64_t n, int64_t ntiles, double *__restrict__ scalars,
    int32_t *__restrict__ anc, Key key, uint32_t t, uint32_t p, int32_t force,
    const double *__restrict__ G, int32_t *__restrict__ counters)
{
    __shared__ double sS[TILE];
    __shared__ double red[NWAVES];
    __shared__ long long rng_lohi[2];
    __shared__ int jstar_sh;
    const int tid = threadIdx.x;
    const bool go = force != 0 || scalars[SMC_S_FLAG] != 0.0;
    const uint4 wU = draw(key, 0, t, TAG_RESAMPLE, 0, p);
    const double U = u53(wU.x, wU.y);
    if (!go) {
        if (blockIdx.x == 0 && tid == 0)
            scalars[SMC_S_RESAMPLED] = 0.0;
        return;
    }
    const int64_t b = blockIdx.x;
    const int64_t base = b * TILE;
    const int len = (int)min((int64_t)TILE, n - base);
    const double M = scalars[SMC_S_M];
    const double stot = prefix[ntiles];
    if (!(stot > 0.0) || !isfinite(stot) || !isfinite(M)) {
        if (b == 0 && tid == 0) {
            atomicOr(&counters[CNT_ERR], SMC_DEVERR_ZERO_WEIGHTS);
            scalars[SMC_S_RESAMPLED] = 0.0;
        }
        return;
    }
    const double Pb = prefix[b], Pb1 = prefix[b + 1];
    const double mb = part[b].m;
    const double sc = mb > -INFINITY ? exp(mb - M) : 0.0;

    double carry = 0.0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + tid;
        double w = 0.0;
        if (i < n) {
            const double l = lw[i];
            w = (l > -INFINITY && mb > -INFINITY) ? exp(l - mb) : 0.0;
        }
        double tot;
        const double incl = block_incl_scan<NWAVES>(w, red, &tot);
        sS[k * TPB + tid] = fmin(Pb + (carry + incl) * sc, Pb1);
        carry += tot;
    }
    __syncthreads();
    if (tid == 0)
        sS[len - 1] = Pb1;
    __syncthreads();

    const bool has_last = Pb < stot && Pb1 >= stot;
    if (SCHEME == SMC_RS_MULTINOMIAL) {
        const MultiPred pred{G, G[n], stot, n};
        if (wave_id() < 2) {
            const double x = wave_id() == 0 ? Pb : Pb1;
            const int64_t cnt = count_below_search(pred, x, n);
            if (lane_id() == 0)
                rng_lohi[wave_id()] = cnt;
        }
    } else if (tid < 2) {
        const double x = tid == 0 ? Pb : Pb1;
        int64_t cnt;
        if (SCHEME == SMC_RS_SYSTEMATIC) {
            const SysPred pred{U, stot, n};
            cnt = count_below_walk(pred, x, n, ceil(x / stot * (double)n - U));
        } else {
            const StratPred pred{key, t, p, stot, n};
            cnt = count_below_walk(pred, x, n, floor(x / stot * (double)n - 0.5));
        }
        rng_lohi[tid] = cnt;
    }
    if (tid == 0) {
        // first element equal to the total: the last positive-weight particle
        int lo = 0, hi = len - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sS[mid] >= stot)
                hi = mid;
            else
                lo = mid + 1;
        }
        jstar_sh = lo;
    }
    __syncthreads();
    const int64_t lo = rng_lohi[0];
    const int64_t hi = has_last ? n : (int64_t)rng_lohi[1];
    const int jstar = jstar_sh;

    for (int64_t i = lo + tid; i < hi; i += TPB) {
        double x;
        if (SCHEME == SMC_RS_SYSTEMATIC)
            x = SysPred{U, stot, n}(i);
        else if (SCHEME == SMC_RS_STRATIFIED)
            x = StratPred{key, t, p, stot, n}(i);
        else
            x = MultiPred{G, G[n], stot, n}(i);
        int l = 0, h = len;  // first j with sS[j] > x
        while (l < h) {
            const int mid = (l + h) >> 1;
            if (sS[mid] > x)
                h = mid;
            else
                l = mid + 1;
        }
        anc[i] = (int32_t)(base + (l < len ? l : jstar));
    }
    if (b == 0 && tid == 0) {
        scalars[SMC_S_RESAMPLED] = 1.0;
        scalars[SMC_S_LPRE] = scalars[SMC_S_L];
        scalars[SMC_S_L] = log((double)n);
        scalars[SMC_S_U] = SCHEME == SMC_RS_SYSTEMATIC ? U : 0.0;
    }
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

__global__ __launch_bounds__(FIN_PASS_TPB) void mn_prefix_kernel(
    const double *__restrict__ scalars, int32_t force, const double *__restrict__ gtile,
    int64_t gtiles, double *__restrict__ gprefix)
{
    __shared__ double sv[FIN_LDS];
    __shared__ double red[FIN_PASS_TPB / WAVE];
    if (!(force != 0 || scalars[SMC_S_FLAG] != 0.0))
        return;
    tile_offsets(gtiles, [&](int64_t b) { return gtile[b]; }, gprefix, sv, red);
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
    const Key key = make_key(c.cfg.seed);
    const uint32_t p = c.cfg.problem_id;
    const dim3 grid((unsigned)c.ntiles);
    switch (c.cfg.scheme) {
    case SMC_RS_SYSTEMATIC:
        hipLaunchKernelGGL(resample_kernel<SMC_RS_SYSTEMATIC>, grid, dim3(TPB), 0, c.stream,
                           c.buf.log_weight, c.partials(), c.prefix(), c.n, c.ntiles,
                           c.buf.scalars, c.buf.ancestors, key, (uint32_t)step, p, force,
                           (const double *)nullptr, c.counters());
        break;
    case SMC_RS_STRATIFIED:
        hipLaunchKernelGGL(resample_kernel<SMC_RS_STRATIFIED>, grid, dim3(TPB), 0, c.stream,
                           c.buf.log_weight, c.partials(), c.prefix(), c.n, c.ntiles,
                           c.buf.scalars, c.buf.ancestors, key, (uint32_t)step, p, force,
                           (const double *)nullptr, c.counters());
        break;
    default: {
        const int64_t count = c.n + 1;
        hipLaunchKernelGGL(mn_tile_sum_kernel, dim3((unsigned)c.gtiles), dim3(TPB), 0, c.stream,
                           c.buf.scalars, force, count, key, (uint32_t)step, p, c.gtile());
        hipLaunchKernelGGL(mn_prefix_kernel, dim3(1), dim3(FIN_PASS_TPB), 0, c.stream, c.buf.scalars,
                           force, c.gtile(), c.gtiles, c.gprefix());
        hipLaunchKernelGGL(mn_write_kernel, dim3((unsigned)c.gtiles), dim3(TPB), 0, c.stream,
                           c.buf.scalars, force, count, key, (uint32_t)step, p, c.gprefix(),
                           c.g());
        hipLaunchKernelGGL(resample_kernel<SMC_RS_MULTINOMIAL>, grid, dim3(TPB), 0, c.stream,
                           c.buf.log_weight, c.partials(), c.prefix(), c.n, c.ntiles,
                           c.buf.scalars, c.buf.ancestors, key, (uint32_t)step, p, force,
                           (const double *)c.g(), c.counters());
    }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Monitors: per-tile sums of w_i and w_i x_r,i (w_i = exp(lw_i - M), or 1
// after a resample), column-major [1 + rows][ntiles], then one workgroup
// combines the tiles in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(TPB) void mon_partial_kernel(
    const T *__restrict__ x, int rows, int64_t n, const double *__restrict__ lw,
    const int32_t *__restrict__ anc, const double *__restrict__ scalars, int gather_check,
    int reset_check, double *__restrict__ mon, int64_t ntiles)
{
    __shared__ double red[NWAVES];
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
            w[k] = reset ? 1.0 : (lw[i] > -INFINITY ? exp(lw[i] - M) : 0.0);
        }
    }
    double sw = w[0] + w[1] + w[2] + w[3];
    sw = block_sum<NWAVES>(sw, red);
    if (threadIdx.x == 0)
        mon[blockIdx.x] = sw;
    for (int r = 0; r < rows; ++r) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            if (w[k] != 0.0)
                s += w[k] * (double)x[(int64_t)r * n + src[k]];
        s = block_sum<NWAVES>(s, red);
        if (threadIdx.x == 0)
            mon[(int64_t)(1 + r) * ntiles + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(FIN_PASS_TPB) void mon_final_kernel(const double *__restrict__ mon,
                                                                 int64_t ntiles, MonDest md,
                                                                 double *__restrict__ hist,
                                                                 int64_t hist_len)
{
    __shared__ double red[FIN_PASS_TPB / WAVE];
    __shared__ double col[MON_STRIDE];
    mon_combine(mon, ntiles, md, hist, hist_len, red, col);
}

hipError_t launch_monitor(Ctx &c, int32_t step, double *out_dev, int rows, bool gather_pending,
                          bool reset_pending)
{
    const dim3 grid((unsigned)c.ntiles);
    if (c.elem_bytes == 4)
        hipLaunchKernelGGL(mon_partial_kernel<float>, grid, dim3(TPB), 0, c.stream,
                           (const float *)c.state_ptr(), rows, c.n, c.buf.log_weight,
                           c.buf.ancestors, c.buf.scalars, (int)gather_pending,
                           (int)reset_pending, c.mon(), c.ntiles);
    else
        hipLaunchKernelGGL(mon_partial_kernel<double>, grid, dim3(TPB), 0, c.stream,
                           (const double *)c.state_ptr(), rows, c.n, c.buf.log_weight,
                           c.buf.ancestors, c.buf.scalars, (int)gather_pending,
                           (int)reset_pending, c.mon(), c.ntiles);
    const MonDest md = mon_dest(c, step, rows, out_dev);
    hipLaunchKernelGGL(mon_final_kernel, dim3(1), dim3(FIN_PASS_TPB), 0, c.stream, c.mon(),
                       c.ntiles, md, c.buf.history, c.buf.history_len);
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
