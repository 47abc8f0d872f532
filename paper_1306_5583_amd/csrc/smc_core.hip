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

// ---------------------------------------------------------------------------
// Cumulative offsets of `count` non-negative tile values v_b in one
// workgroup of FIN_TPB lanes: out[b] = sum_{b' < b} v_b', out[count] = total.
// Passes of FIN_PASS values; in a pass lane t owns the FIN_IT consecutive
// values starting at FIN_IT t (all loaded at once), sums them sequentially,
// the lane totals are scanned across the workgroup in a fixed order, and an
// exact running maximum keeps out[] non-decreasing.  The same inputs always
// give the same outputs.  `val(b)` is called exactly once per b, in
// increasing b for each lane.
// ---------------------------------------------------------------------------
constexpr int FIN_TPB = 512;
constexpr int FIN_NW = FIN_TPB / WAVE;
constexpr int FIN_IT = 8;
constexpr int FIN_PASS = FIN_TPB * FIN_IT;

// One pass: lane values v[] for b0 .. b0+FIN_IT-1; returns the new carry.
__device__ __forceinline__ double offsets_pass(const double (&v)[FIN_IT], int64_t b0,
                                               int64_t count, double carry, double *out,
                                               double *red)
{
    double e[FIN_IT];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        e[k] = run;
        run += v[k];
    }
    double total;
    const double excl = block_excl_scan<FIN_NW>(run, red, &total);
    double last = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        e[k] = carry + (excl + e[k]);
        last = fmax(last, e[k]);
    }
    const double incl_max = block_incl_max_scan<FIN_NW>(last, red);
    double floor_v = lane_prev(incl_max, 0.0);
    __syncthreads();
    if (lane_id() == WAVE - 1)
        red[wave_id()] = incl_max;
    __syncthreads();
    if (lane_id() == 0)
        floor_v = wave_id() == 0 ? carry : red[wave_id() - 1];
    floor_v = fmax(floor_v, carry);
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k)
        if (b0 + k < count)
            out[b0 + k] = fmax(e[k], floor_v);
    const double pass_max = red[FIN_NW - 1];
    __syncthreads();
    return fmax(carry + total, pass_max);
}

template <typename F>
__device__ double tile_offsets(int64_t count, F val, double *out, double *red)
{
    double carry = 0.0;
    for (int64_t pbase = 0; pbase < count; pbase += FIN_PASS) {
        const int64_t b0 = pbase + (int64_t)threadIdx.x * FIN_IT;
        double v[FIN_IT];
#pragma unroll
        for (int k = 0; k < FIN_IT; ++k)
            v[k] = b0 + k < count ? val(b0 + k) : 0.0;
        carry = offsets_pass(v, b0, count, carry, out, red);
    }
    if (threadIdx.x == 0)
        out[count] = carry;
    return carry;
}

// ---------------------------------------------------------------------------
// Normalisation and the completion of monitor partials.  A move can carry
// the monitor partials of the previous step (per tile: sum w and sum w x
// for each monitored row); their importance-sampling estimates are
// completed alongside the next normalisation.
// ---------------------------------------------------------------------------
struct MonDest {
    int32_t step;     // history row, or -1 when no monitor partials are pending
    int rows;         // monitored rows (partial columns 1..rows; column 0 = sum w)
    int hist_col;     // first history column receiving estimates
    int hist_ncols;   // how many of the last rows go to the history
    double *out;      // optional device output [rows]
    double *scalars;  // mixture sampler: path-sampling accumulator (else null)
    double alpha;     // tempering exponent of the monitored particles
};

// Sums the tile partials of every monitored row with the whole workgroup:
// thread t adds tiles t, t + NTHR, t + 2 NTHR, ... in order (MON_IT of them
// loaded at once, two rows at a time), each wave adds its lanes, and thread r
// adds the NW wave sums of row r in wave order, so the result does not depend
// on timing.  `red` holds MON_STRIDE * NW doubles, `col` MON_STRIDE.
constexpr int MON_IT = 8;
template <int NTHR>
__device__ void mon_combine(const double *__restrict__ mon, int64_t ntiles, const MonDest &d,
                            double *__restrict__ hist, int64_t hist_len, double *red,
                            double *col)
{
    constexpr int NW = NTHR / WAVE;
    const int tid = threadIdx.x, w = wave_id();
    if (ntiles <= NTHR) {
        // one tile per thread: up to 16 rows' loads in flight per round
        // (the same sums in the same order as below)
        constexpr int RG = 16;
        for (int r0 = 0; r0 <= d.rows; r0 += RG) {
            double x[RG];
#pragma unroll
            for (int g = 0; g < RG; ++g)
                x[g] = (r0 + g <= d.rows && tid < ntiles) ? mon[(int64_t)(r0 + g) * ntiles + tid]
                                                          : 0.0;
#pragma unroll
            for (int g = 0; g < RG; ++g)
                if (r0 + g <= d.rows) {
                    const double v = wave_sum(x[g]);
                    if (lane_id() == 0)
                        red[(r0 + g) * NW + w] = v;
                }
        }
    }
    for (int r0 = 0; ntiles > NTHR && r0 <= d.rows; r0 += 2) {
        const bool two = r0 + 1 <= d.rows;
        const double *m0 = mon + (int64_t)r0 * ntiles;
        const double *m1 = two ? m0 + ntiles : m0;
        double a0 = 0.0, a1 = 0.0;
        for (int64_t base = 0; base < ntiles; base += (int64_t)MON_IT * NTHR) {
            double x0[MON_IT], x1[MON_IT];
#pragma unroll
            for (int k = 0; k < MON_IT; ++k) {
                const int64_t b = base + (int64_t)k * NTHR + tid;
                x0[k] = b < ntiles ? m0[b] : 0.0;
                x1[k] = b < ntiles ? m1[b] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < MON_IT; ++k) {
                a0 += x0[k];
                a1 += x1[k];
            }
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane_id() == 0) {
            red[r0 * NW + w] = a0;
            if (two)
                red[(r0 + 1) * NW + w] = a1;
        }
    }
    __syncthreads();
    if (tid <= d.rows) {
        double a = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v)
            a += red[tid * NW + v];
        col[tid] = a;
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
        // path sampling (Section 5.2): the last row is U = sum W l at alpha;
        // one trapezoid from the previously monitored (alpha, U)
        if (d.scalars && r == d.rows - 1) {
            double *sc = d.scalars;
            const double a0 = sc[SMC_S_PS_ALPHA];
            double ps = sc[SMC_S_PS_LOGZ];
            if (a0 >= 0.0)
                ps += 0.5 * (d.alpha - a0) * (est + sc[SMC_S_PS_U]);
            sc[SMC_S_PS_LOGZ] = ps;
            sc[SMC_S_PS_U] = est;
            sc[SMC_S_PS_ALPHA] = d.alpha;
            if (hist && d.step >= 0 && d.step < hist_len)
                hist[(int64_t)d.step * SMC_HIST_COLS + SMC_H_PS] = ps;
        }
    }
}

constexpr int FIN_MON_ROWS = 4;  // rows a move can carry (the tracking state)

// Single pass over at most FIN_PASS tile partials.  The partials are read
// coalesced (lane t of the workgroup takes tiles t, t + FIN_TPB, ...), the
// scaled tile weights s1 exp(m - M) go through LDS, and lane t then owns the
// FIN_IT consecutive tiles from FIN_IT t.  (Reading each lane's consecutive
// 256 bytes directly touches every cache line from FIN_IT lanes' loads and
// thrashes the vector L1 once the partials outgrow it.)  The cumulative
// offsets are the lane's running sums on top of the workgroup scan of the
// lane totals, each clamped to the lane's inclusive value, which is exactly
// the next lane's starting offset (and the next wave's: the wave totals are
// summed in order), so the offsets never decrease; they return through LDS
// for coalesced stores.  The sum of squares rides on the same barrier pair.
// LDS slot of tile b: one pad double after every FIN_IT (two-way bank
// conflicts at most on both the strided writes and the consecutive reads).
__device__ __forceinline__ int fin_slot(int b) { return b + b / FIN_IT; }
constexpr int FIN_LDS = FIN_PASS + FIN_PASS / FIN_IT;

__device__ __forceinline__ void normalise_one_pass(const TilePartial *__restrict__ part,
                                                   int64_t ntiles, double *__restrict__ prefix,
                                                   double *red, double *wl, double *M_out,
                                                   double *S1_out, double *S2_out)
{
    const int tid = threadIdx.x;
    TilePartial q[FIN_IT];
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        const int64_t b = (int64_t)k * FIN_TPB + tid;
        q[k] = b < ntiles ? part[b] : TilePartial{-INFINITY, 0.0, 0.0, 0.0};
    }
    double m = -INFINITY;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k)
        m = fmax(m, q[k].m);
    const double M = block_max<FIN_NW>(m, red);
    double s2 = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        const double sc = q[k].m > -INFINITY ? exp_nonpos_d(q[k].m - M) : 0.0;
        wl[fin_slot(k * FIN_TPB + tid)] = q[k].s1 * sc;
        s2 += q[k].s2 * (sc * sc);
    }
    __syncthreads();
    double e[FIN_IT];
    double run = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        e[k] = run;
        run += wl[fin_slot(tid * FIN_IT + k)];
    }
    const double incl = wave_incl_scan(run);
    const double excl = lane_prev(incl, 0.0);
    const double s2w = wave_sum(s2);
    __syncthreads();  // red is reused from block_max
    if (lane_id() == WAVE - 1) {
        red[wave_id()] = incl;
        red[FIN_NW + wave_id()] = s2w;
    }
    __syncthreads();
    double before = 0.0, total = 0.0, S2 = 0.0;
#pragma unroll
    for (int w = 0; w < FIN_NW; ++w) {
        if (w < wave_id())
            before += red[w];
        total += red[w];
        S2 += red[FIN_NW + w];
    }
    const double lo = lane_id() == 0 ? before : before + excl;
    const double hi = before + incl;
    // back through LDS (its reads above completed before the two barriers)
    // for coalesced stores
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k)
        wl[fin_slot(tid * FIN_IT + k)] = fmin(lo + e[k], hi);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        const int64_t b = (int64_t)k * FIN_TPB + tid;
        if (b < ntiles)
            prefix[b] = wl[fin_slot(k * FIN_TPB + tid)];
    }
    if (tid == 0)
        prefix[ntiles] = total;
    *M_out = M;
    *S1_out = total;
    *S2_out = S2;
}

// Normalisation (one workgroup): global max M, tile offsets of the
// cumulative weights, S1 = sum exp(lw - M), S2 = sum exp(2 (lw - M)),
// L = M + log S1, L2 = 2M + log S2, ESS = exp(2L - L2), dlogZ = L - L_prev,
// decision ESS < tau N (tau >= 1 always, tau <= 0 never).
__device__ __forceinline__ void normalise_block(const Prob &P, int32_t step)
{
    __shared__ double red[2 * FIN_NW];
    __shared__ double wl[FIN_LDS];
    const TilePartial *__restrict__ part = P.partials;
    const int64_t ntiles = P.ntiles, n = P.n;
    double *__restrict__ prefix = P.prefix;
    double *__restrict__ scalars = P.scalars;
    const int tid = threadIdx.x;
    // the previous L and log Z, fetched while the partials arrive
    double Lprev = 0.0, logz_prev = 0.0;
    if (tid == 0) {
        Lprev = scalars[SMC_S_L];
        logz_prev = scalars[SMC_S_LOGZ];
    }
    double M, S1, S2;
    if (ntiles <= FIN_PASS) {
        normalise_one_pass(part, ntiles, prefix, red, wl, &M, &S1, &S2);
    } else {
        double m = -INFINITY;
        for (int64_t b = (int64_t)tid * FIN_IT; b < ntiles; b += FIN_PASS) {
            double qm[FIN_IT];
#pragma unroll
            for (int k = 0; k < FIN_IT; ++k)
                qm[k] = b + k < ntiles ? part[b + k].m : -INFINITY;
#pragma unroll
            for (int k = 0; k < FIN_IT; ++k)
                m = fmax(m, qm[k]);
        }
        M = block_max<FIN_NW>(m, red);
        double s2 = 0.0;
        S1 = tile_offsets(
            ntiles,
            [&](int64_t b) {
                const TilePartial q = part[b];
                const double sc = q.m > -INFINITY ? exp_nonpos_d(q.m - M) : 0.0;
                s2 += q.s2 * (sc * sc);
                return q.s1 * sc;
            },
            prefix, red);
        S2 = block_sum<FIN_NW>(s2, red);
    }
    if (tid == 0) {
        const double threshold = P.threshold;
        const double L = M + log(S1);
        const double L2 = 2.0 * M + log(S2);
        const double ess = exp(2.0 * L - L2);
        const double dlogz = L - Lprev;
        const double logz = logz_prev + dlogz;
        int flag;
        if (threshold >= 1.0)
            flag = 1;
        else if (threshold <= 0.0)
            flag = 0;
        else
            flag = ess < threshold * (double)n;
        if (!(S1 > 0.0) || !isfinite(S1) || !isfinite(M)) {
            atomicOr(&P.counters[CNT_ERR], SMC_DEVERR_NONFINITE);
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
        if (P.hist && step >= 0 && step < P.hist_len) {
            double *h = P.hist + (int64_t)step * SMC_HIST_COLS;
            h[SMC_H_ESS] = ess;
            h[SMC_H_FLAG] = (double)flag;
            h[SMC_H_DLOGZ] = dlogz;
            h[SMC_H_LOGZ] = logz;
            h[SMC_H_L] = L;
        }
    }
}

// Completion of monitor partials carried by a move (importance-sampling
// estimates of the previous step), independent of the normalisation.
__device__ __forceinline__ void monitor_block(const Prob &P, const MonDest &md)
{
    __shared__ double red[MON_STRIDE * FIN_NW];
    __shared__ double col[MON_STRIDE];
    mon_combine<FIN_TPB>(P.mon, P.ntiles, md, P.hist, P.hist_len, red, col);
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

// Cumulative weights of one tile in the blocked arrangement: lane t owns the
// four consecutive particles base + 4t .. base + 4t + 3.  Returns S for those
// four and, in s_prev, S of the particle before the first (Pb for lane 0).
// S is clamped into [Pb, Pb1] and, from the tile's last positive-weight
// particle on, equals Pb1 exactly, so consecutive tiles join without gaps or
// overlaps and a zero-weight particle never owns a slot.
struct TileCdf {
    double S[ITEMS];
    double s_prev;
    int lastpos;  // tile-local index of the last positive-weight particle, -1 if none
};

// The lane's ITEMS log-weights of the tile (-inf past its end).
__device__ __forceinline__ void tile_load_lw(const double *__restrict__ lw, int64_t base, int len,
                                             double (&l)[ITEMS])
{
    const int j0 = ITEMS * threadIdx.x;
    if (j0 + ITEMS <= len) {
        const double4 q = *reinterpret_cast<const double4 *>(lw + base + j0);
        l[0] = q.x;
        l[1] = q.y;
        l[2] = q.z;
        l[3] = q.w;
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            l[k] = j0 + k < len ? lw[base + j0 + k] : -INFINITY;
    }
}

__device__ __forceinline__ TileCdf tile_cdf(const double (&l)[ITEMS], double mb, double sc,
                                            double Pb, double Pb1, double *red,
                                            double *wave_last, int *wave_pos)
{
    const int tid = threadIdx.x;
    const int j0 = ITEMS * tid;
    double a[ITEMS];
    double run = 0.0;
    int lastpos = -1;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const double w = mb > -INFINITY ? exp_nonpos_d(l[k] - mb) : 0.0;
        run += w;
        a[k] = run;
        lastpos = w > 0.0 ? j0 + k : lastpos;
    }
    lastpos = wave_max_i(lastpos);
    if (lane_id() == 0)
        wave_pos[wave_id()] = lastpos;
    double total;
    const double excl = block_excl_scan<NWAVES>(run, red, &total);  // synchronises
#pragma unroll
    for (int w = 0; w < NWAVES; ++w)
        lastpos = max(lastpos, wave_pos[w]);
    TileCdf r;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int j = j0 + k;
        r.S[k] = j < lastpos ? fmin(Pb + (excl + a[k]) * sc, Pb1) : Pb1;
    }
    if (lastpos < 0) {  // no positive weight in the tile: Pb == Pb1
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
            r.S[k] = Pb;
    }
    // S of the previous particle: the neighbouring lane's last value
    double prev = lane_prev(r.S[ITEMS - 1], 0.0);
    __syncthreads();
    if (lane_id() == WAVE - 1)
        wave_last[wave_id()] = r.S[ITEMS - 1];
    __syncthreads();
    if (lane_id() == 0)
        prev = wave_id() == 0 ? Pb : wave_last[wave_id() - 1];
    r.s_prev = prev;
    r.lastpos = lastpos;
    return r;
}

// Sorted ancestors of one tile by a merge of two sorted sequences: the
// tile's cumulative weights S_j and the ordered uniforms u_i of the slots it
// owns, [c(Pb), c(Pb1)) with c(x) = #{i : u_i S < x} (to N for the tile
// holding the last positive weight).  Slot i goes to the first j with
// S_j > u_i S.  Each lane takes an equal share of the merged sequence,
// finds its start by a merge-path search, then walks it: the work is
// balanced however unevenly the slots fall on the particles.  Slot uniforms
// are staged in LDS when the tile owns at most RS_UCAP slots.
constexpr int RS_UCAP = 2048;

template <int SCHEME>
__device__ __forceinline__ void resample_tile(const Prob &P, int64_t b, uint32_t t, int32_t force,
                                              const double *__restrict__ G)
{
    const double *__restrict__ lw = P.lw;
    const TilePartial *__restrict__ part = P.partials;
    const double *__restrict__ prefix = P.prefix;
    const int64_t n = P.n, ntiles = P.ntiles;
    double *__restrict__ scalars = P.scalars;
    int32_t *__restrict__ anc = P.anc;
    const Key key = P.key;
    const uint32_t p = P.problem_id;
    int32_t *__restrict__ counters = P.counters;
    __shared__ double sS[TILE];
    __shared__ double sU[RS_UCAP];
    __shared__ double red[NWAVES];
    __shared__ double wave_last[NWAVES];
    __shared__ int wave_pos[NWAVES];
    __shared__ long long rng_lohi[2];
    const int tid = threadIdx.x;
    const bool go = force != 0 || scalars[SMC_S_FLAG] != 0.0;
    const uint4 wU = draw(key, 0, t, TAG_RESAMPLE, 0, p);
    const double U = u53(wU.x, wU.y);
    if (!go) {
        if (b == 0 && tid == 0)
            scalars[SMC_S_RESAMPLED] = 0.0;
        return;
    }
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
    const double sc = mb > -INFINITY ? exp_nonpos_d(mb - M) : 0.0;
    double l[ITEMS];
    tile_load_lw(lw, base, len, l);
    const TileCdf cdf = tile_cdf(l, mb, sc, Pb, Pb1, red, wave_last, wave_pos);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        sS[ITEMS * tid + k] = cdf.S[k];

    const SysPred sys{U, stot, n};
    const StratPred strat{key, t, p, stot, n};
    const MultiPred multi{G, SCHEME == SMC_RS_MULTINOMIAL ? G[n] : 1.0, stot, n};
    auto pred = [&](int64_t i) -> double {
        if (SCHEME == SMC_RS_SYSTEMATIC)
            return sys(i);
        if (SCHEME == SMC_RS_STRATIFIED)
            return strat(i);
        return multi(i);
    };
    const double nd = (double)n;
    if (SCHEME == SMC_RS_MULTINOMIAL) {
        if (wave_id() < 2) {
            const int64_t cnt = count_below_search(multi, wave_id() == 0 ? Pb : Pb1, n);
            if (lane_id() == 0)
                rng_lohi[wave_id()] = cnt;
        }
    } else if (tid < 2) {
        const double x = tid == 0 ? Pb : Pb1;
        rng_lohi[tid] = SCHEME == SMC_RS_SYSTEMATIC
                            ? count_below_walk(sys, x, n, ceil(x / stot * nd - U))
                            : count_below_walk(strat, x, n, floor(x / stot * nd - 0.5));
    }
    __syncthreads();
    const bool has_last = Pb < stot && Pb1 >= stot;
    const int64_t lo = rng_lohi[0];
    const int64_t hi = has_last ? n : max((int64_t)rng_lohi[1], lo);
    const int64_t ns = hi - lo;
    const int jstar = cdf.lastpos < 0 ? 0 : cdf.lastpos;
    const bool staged = ns <= RS_UCAP;
    if (staged)
        for (int64_t q = tid; q < ns; q += TPB)
            sU[q] = pred(lo + q);
    __syncthreads();
    auto u_at = [&](int64_t q) -> double { return staged ? sU[q] : pred(lo + q); };

    const int64_t total = (int64_t)len + ns;
    const int64_t ipt = ceil_div(total, TPB);
    const int64_t d0 = min((int64_t)tid * ipt, total);
    const int64_t d1 = min(d0 + ipt, total);
    // merge-path split of the first d0 items: owners consumed = first j with
    // S_j not preceding slot d0-1-j  (an owner precedes a slot iff S_j <= u)
    int64_t jl = max((int64_t)0, d0 - ns), jh = min(d0, (int64_t)len);
    while (jl < jh) {
        const int64_t mid = (jl + jh) >> 1;
        if (sS[mid] <= u_at(d0 - 1 - mid))
            jl = mid + 1;
        else
            jh = mid;
    }
    int64_t j = jl, i = d0 - jl;
    double uj = i < ns ? u_at(i) : 0.0;
    for (int64_t s = d0; s < d1; ++s) {
        if (j < len && (i >= ns || sS[j] <= uj)) {
            ++j;
        } else {
            anc[lo + i] = (int32_t)(base + (j < len ? j : jstar));
            ++i;
            if (i < ns)
                uj = u_at(i);
        }
    }
    if (b == 0 && tid == 0) {
        scalars[SMC_S_RESAMPLED] = 1.0;
        scalars[SMC_S_LPRE] = scalars[SMC_S_L];
        scalars[SMC_S_L] = log(nd);
        scalars[SMC_S_U] = SCHEME == SMC_RS_SYSTEMATIC ? U : 0.0;
    }
}

// Systematic resampling of one tile by replication numbers (Section 2.1:
// particle j copied R_j times, sum N).  Particle j owns the slots
// [c(S_{j-1}), c(S_j)) with c(x) = min(N, max(0, ceil(x N / S - U))) (one
// fused multiply-add), the number of ordered uniforms (i + U) / N below
// x / S, so R_j = c(S_j) - c(S_{j-1}) and every lane finds the ranges of its
// own particles directly.  The tile's slots are then
// filled through LDS in chunks of RS_UCAP: each particle with a non-empty
// range marks the range's first slot with its index and an inclusive
// max-scan spreads it over the range, which keeps the stores coalesced and
// the work even however the slots fall on the particles.
__device__ __forceinline__ void resample_sys_tile(const Prob &P, int64_t b, uint32_t t,
                                                  int32_t force)
{
    constexpr int QPT = RS_UCAP / TPB;  // chunk slots per lane
    const double *__restrict__ lw = P.lw;
    const double *__restrict__ prefix = P.prefix;
    const int64_t n = P.n, ntiles = P.ntiles;
    double *__restrict__ scalars = P.scalars;
    int32_t *__restrict__ anc = P.anc;
    __shared__ double red[NWAVES];
    __shared__ double wave_last[NWAVES];
    __shared__ int wave_pos[NWAVES];
    __shared__ int wave_end[NWAVES];
    __shared__ int wave_max[NWAVES];
    __shared__ int owner[RS_UCAP];
    __shared__ long long tile_lo;
    __shared__ double sh_U;
    const int tid = threadIdx.x;
    const int64_t base = b * TILE;
    const int len = (int)min((int64_t)TILE, n - base);
    // every load of the tile in one round trip: the decision, the
    // normalisation and the log-weights (the last read in vain on steps that
    // do not resample)
    const double flag = scalars[SMC_S_FLAG];
    const double M = scalars[SMC_S_M];
    const double stot = prefix[ntiles];
    const double Pb = prefix[b], Pb1 = prefix[b + 1];
    const double mb = P.partials[b].m;
    double l[ITEMS];
    tile_load_lw(lw, base, len, l);
    const bool go = force != 0 || flag != 0.0;
    if (!go) {
        if (b == 0 && tid == 0)
            scalars[SMC_S_RESAMPLED] = 0.0;
        return;
    }
    if (!(stot > 0.0) || !isfinite(stot) || !isfinite(M)) {
        if (b == 0 && tid == 0) {
            atomicOr(&P.counters[CNT_ERR], SMC_DEVERR_ZERO_WEIGHTS);
            scalars[SMC_S_RESAMPLED] = 0.0;
        }
        return;
    }
    const double sc = mb > -INFINITY ? exp_nonpos_d(mb - M) : 0.0;
    // the step's systematic offset: one lane draws it while the tile loads
    if (tid == 0) {
        const uint4 wU = draw(P.key, 0, t, TAG_RESAMPLE, 0, P.problem_id);
        sh_U = u53(wU.x, wU.y);
    }
    const TileCdf cdf = tile_cdf(l, mb, sc, Pb, Pb1, red, wave_last, wave_pos);
    const double U = sh_U;  // tile_cdf ends on a barrier
    const double nd = (double)n;
    const double r = nd / stot;
    // c(x) = min(N, max(0, ceil(x N / S - U))): the number of uniforms
    // (i + U) / N below x / S, in closed form
    auto count = [&](double x) -> int64_t {
        const double c = ceil(fma(x, r, -U));
        return !(c > 0.0) ? 0 : (c >= nd ? n : (int64_t)c);
    };
    // the tile holding the last positive weight also takes the slots whose
    // uniform reaches the total (from its last positive particle on)
    const bool has_last = Pb < stot && Pb1 >= stot;
    const int j0 = ITEMS * tid;
    int ce[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        ce[k] = (int)((has_last && j0 + k >= cdf.lastpos) ? n : count(cdf.S[k]));
    if (tid == 0)
        tile_lo = count(Pb);
    int cs0 = dpp::mov_i<dpp::WAVE_SHR1>(ce[ITEMS - 1], 0);
    if (lane_id() == WAVE - 1)
        wave_end[wave_id()] = ce[ITEMS - 1];
    __syncthreads();
    if (lane_id() == 0)
        cs0 = wave_id() == 0 ? (int)tile_lo : wave_end[wave_id() - 1];
    const int64_t lo = tile_lo, hi = wave_end[NWAVES - 1];
    int carry = -1;
    for (int64_t c0 = lo; c0 < hi; c0 += RS_UCAP) {
        const int cn = (int)min((int64_t)RS_UCAP, hi - c0);
#pragma unroll
        for (int i = 0; i < QPT; ++i)
            owner[tid + i * TPB] = -1;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int st = k == 0 ? cs0 : ce[k - 1];
            if (ce[k] > st && st >= c0 && st < c0 + cn)
                owner[st - c0] = j0 + k;
        }
        __syncthreads();
        // inclusive max-scan of owner[0, cn): QPT consecutive slots per lane
        int v[QPT];
        int run = -1;
#pragma unroll
        for (int i = 0; i < QPT; ++i) {
            run = max(run, owner[tid * QPT + i]);
            v[i] = run;
        }
        const int incl = dpp::incl_scan_i(run, -1, OpMaxI{});
        int before = dpp::mov_i<dpp::WAVE_SHR1>(incl, -1);
        if (lane_id() == WAVE - 1)
            wave_max[wave_id()] = incl;
        __syncthreads();
        for (int w = 0; w < wave_id(); ++w)
            before = max(before, wave_max[w]);
        before = max(before, carry);
        int last = carry;
#pragma unroll
        for (int w = 0; w < NWAVES; ++w)
            last = max(last, wave_max[w]);
#pragma unroll
        for (int i = 0; i < QPT; ++i)
            owner[tid * QPT + i] = max(v[i], before);
        __syncthreads();
        for (int q = tid; q < cn; q += TPB)
            anc[c0 + q] = (int32_t)(base + owner[q]);
        carry = last;
        __syncthreads();
    }
    if (b == 0 && tid == 0) {
        scalars[SMC_S_RESAMPLED] = 1.0;
        scalars[SMC_S_LPRE] = scalars[SMC_S_L];
        scalars[SMC_S_L] = log(nd);
        scalars[SMC_S_U] = U;
    }
}

__global__ __launch_bounds__(TPB) void resample_sys_kernel(Prob P, uint32_t t, int32_t force)
{
    resample_sys_tile(P, blockIdx.x, t, force);
}

template <int SCHEME>
__global__ __launch_bounds__(TPB) void resample_merge_kernel(Prob P, uint32_t t, int32_t force,
                                                             const double *__restrict__ G)
{
    resample_tile<SCHEME>(P, blockIdx.x, t, force, G);
}

// Batched systematic resampling over the tiles of many problems.
__global__ __launch_bounds__(TPB) void resample_batch_kernel(const Prob *__restrict__ probs,
                                                             const int2 *__restrict__ map,
                                                             const int32_t *__restrict__ step)
{
    const int2 pm = map[blockIdx.x];
    resample_sys_tile(probs[pm.x], pm.y, (uint32_t)*step, 0);
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
