// smc_tiles.hpp -- per-tile device functions of the sweep shared by the
// single-problem kernels, the per-phase batched kernels and the persistent
// batched step: normalisation (log-sum-exp, ESS, normalising constant,
// resampling decision, cumulative-weight tile offsets), monitor completion,
// resampling to sorted ancestors, the tracking filter's fused move + weight
// and the mixture sampler's tempering reweight.
#pragma once

#include <math.h>

#include "smc_internal.hpp"

namespace smc {

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
// NT lanes (FIN_TPB unless a caller runs with fewer).
template <int NT = FIN_TPB>
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
    const double excl = block_excl_scan<NT / WAVE>(run, red, &total);
    double last = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        e[k] = carry + (excl + e[k]);
        last = fmax(last, e[k]);
    }
    const double incl_max = block_incl_max_scan<NT / WAVE>(last, red);
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
    const double pass_max = red[NT / WAVE - 1];
    __syncthreads();
    return fmax(carry + total, pass_max);
}

template <int NT = FIN_TPB, typename F>
__device__ double tile_offsets(int64_t count, F val, double *out, double *red)
{
    double carry = 0.0;
    for (int64_t pbase = 0; pbase < count; pbase += NT * FIN_IT) {
        const int64_t b0 = pbase + (int64_t)threadIdx.x * FIN_IT;
        double v[FIN_IT];
#pragma unroll
        for (int k = 0; k < FIN_IT; ++k)
            v[k] = b0 + k < count ? val(b0 + k) : 0.0;
        carry = offsets_pass<NT>(v, b0, count, carry, out, red);
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
template <int NT>
constexpr int fin_lds() { return NT * FIN_IT + NT; }

template <int NT = FIN_TPB>
__device__ __forceinline__ void normalise_one_pass(const TilePartial *__restrict__ part,
                                                   int64_t ntiles, double *__restrict__ prefix,
                                                   double *red, double *wl, double *M_out,
                                                   double *S1_out, double *S2_out)
{
    const int tid = threadIdx.x;
    TilePartial q[FIN_IT];
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        const int64_t b = (int64_t)k * NT + tid;
        q[k] = b < ntiles ? part[b] : TilePartial{-INFINITY, 0.0, 0.0, 0.0};
    }
    double m = -INFINITY;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k)
        m = fmax(m, q[k].m);
    const double M = block_max<(NT / WAVE)>(m, red);
    double s2 = 0.0;
#pragma unroll
    for (int k = 0; k < FIN_IT; ++k) {
        const double sc = q[k].m > -INFINITY ? exp_nonpos_d(q[k].m - M) : 0.0;
        wl[fin_slot(k * NT + tid)] = q[k].s1 * sc;
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
        red[(NT / WAVE) + wave_id()] = s2w;
    }
    __syncthreads();
    double before = 0.0, total = 0.0, S2 = 0.0;
#pragma unroll
    for (int w = 0; w < (NT / WAVE); ++w) {
        if (w < wave_id())
            before += red[w];
        total += red[w];
        S2 += red[(NT / WAVE) + w];
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
        const int64_t b = (int64_t)k * NT + tid;
        if (b < ntiles)
            prefix[b] = wl[fin_slot(k * NT + tid)];
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
template <int NT = FIN_TPB>
__device__ __forceinline__ void normalise_block(const Prob &P, int32_t step)
{
    __shared__ double red[2 * (NT / WAVE)];
    __shared__ double wl[fin_lds<NT>()];
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
    if (ntiles <= (NT * FIN_IT)) {
        normalise_one_pass<NT>(part, ntiles, prefix, red, wl, &M, &S1, &S2);
    } else {
        double m = -INFINITY;
        for (int64_t b = (int64_t)tid * FIN_IT; b < ntiles; b += (NT * FIN_IT)) {
            double qm[FIN_IT];
#pragma unroll
            for (int k = 0; k < FIN_IT; ++k)
                qm[k] = b + k < ntiles ? part[b + k].m : -INFINITY;
#pragma unroll
            for (int k = 0; k < FIN_IT; ++k)
                m = fmax(m, qm[k]);
        }
        M = block_max<(NT / WAVE)>(m, red);
        double s2 = 0.0;
        S1 = tile_offsets<NT>(
            ntiles,
            [&](int64_t b) {
                const TilePartial q = part[b];
                const double sc = q.m > -INFINITY ? exp_nonpos_d(q.m - M) : 0.0;
                s2 += q.s2 * (sc * sc);
                return q.s1 * sc;
            },
            prefix, red);
        S2 = block_sum<(NT / WAVE)>(s2, red);
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
template <int NT = FIN_TPB>
__device__ __forceinline__ void monitor_block(const Prob &P, const MonDest &md)
{
    __shared__ double red[MON_STRIDE * (NT / WAVE)];
    __shared__ double col[MON_STRIDE];
    mon_combine<NT>(P.mon, P.ntiles, md, P.hist, P.hist_len, red, col);
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

// sS (TILE doubles) and sU (RS_UCAP doubles) are the caller's LDS.
template <int SCHEME>
__device__ __forceinline__ void resample_tile(const Prob &P, int64_t b, uint32_t t, int32_t force,
                                              const double *__restrict__ G, double *sS,
                                              double *sU)
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

// One move of Algorithm "pf" for the particles of one tile, reading through
// the pending ancestors, writing the ping-pong partner; with FUSE the
// incremental log-weight of observation y is added (after a resample the
// previous weights count as zero) and the tile partial is produced.  With
// MON the tile also sums w_i and w_i x_i of the incoming population (the
// monitor of the previous step: w_i = 1 after a resample, else
// exp(lw_i - M)), column-major into mon[5][ntiles].
template <typename T, bool FUSE, bool MON>
__device__ __forceinline__ void pf_move_tile(const Prob &P, const T *__restrict__ xin,
                                             T *__restrict__ xout, int64_t tile, uint32_t t,
                                             const double *__restrict__ y, bool gather_check,
                                             bool reset_check)
{
    __shared__ double red[NWAVES];
    const int64_t n = P.n;
    double *__restrict__ lw = P.lw;
    const int32_t *__restrict__ anc = P.anc;
    const bool resampled =
        (gather_check || reset_check) ? P.scalars[SMC_S_RESAMPLED] != 0.0 : false;
    const bool gather = gather_check && resampled;
    const bool reset = reset_check && resampled;
    const int64_t base = tile * TILE;
    const Key key = P.key;
    const uint32_t p = P.problem_id;
    const Motion mv = P.mv;
    const ObsModel obs = P.obs;
    double yx = 0.0, yy = 0.0;
    if (FUSE) {
        yx = y[0];
        yy = y[1];
    }
    const double M = MON ? P.scalars[SMC_S_M] : 0.0;
    double ms[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        const int64_t src = gather ? (int64_t)anc[i] : i;
        const T px = xin[src], py = xin[n + src], vx = xin[2 * n + src], vy = xin[3 * n + src];
        const double lw_in = (FUSE && !reset) || (MON && !reset) ? lw[i] : 0.0;
        if (MON) {
            const double w = reset ? 1.0 : exp_nonpos_d(lw_in - M);
            if (w != 0.0) {
                ms[0] += w;
                ms[1] += w * (double)px;
                ms[2] += w * (double)py;
                ms[3] += w * (double)vx;
                ms[4] += w * (double)vy;
            }
        }
        T npx, npy, nvx, nvy;
        if constexpr (sizeof(T) == 8) {
            const double2 a = normal2(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 0, p));
            const double2 b = normal2(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 1, p));
            npx = (px + mv.dt * vx) + mv.sd_pos * a.x;
            npy = (py + mv.dt * vy) + mv.sd_pos * a.y;
            nvx = vx + mv.sd_vel * b.x;
            nvy = vy + mv.sd_vel * b.y;
        } else {
            const float4 z = normal4f(draw(key, (uint32_t)i, t, TAG_PF_MOVE, 0, p));
            const float dt = (float)mv.dt, sp = (float)mv.sd_pos, sv = (float)mv.sd_vel;
            npx = (px + dt * vx) + sp * z.x;
            npy = (py + dt * vy) + sp * z.y;
            nvx = vx + sv * z.z;
            nvy = vy + sv * z.w;
        }
        xout[i] = npx;
        xout[n + i] = npy;
        xout[2 * n + i] = nvx;
        xout[3 * n + i] = nvy;
        if (FUSE) {
            const double inc = obs((double)npx, yx, (double)npy, yy);
            const double l = lw_in + inc;
            lw[i] = l;
            lwv[k] = l;
        }
    }
    if (FUSE)
        tile_partial(lwv, P.partials + tile, red);
    if (MON) {
        __shared__ double red5[5 * NWAVES];
        block_sum_n<NWAVES, 5>(ms, red5);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int r = 0; r < 5; ++r)
                P.mon[(int64_t)r * P.ntiles + tile] = ms[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Reweighting of Algorithm "gmm": lw <- (reset ? 0 : lw) + dalpha * l, with
// dalpha == 0 adding exactly 0; per-tile partials for the normalisation.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gmm_reweight_tile(const Prob &P, const double *__restrict__ llrow,
                                                  int64_t tile, int reset_check, double dalpha)
{
    __shared__ double red[NWAVES];
    double *__restrict__ lw = P.lw;
    const int64_t n = P.n;
    TilePartial *__restrict__ part = P.partials;
    const bool reset = reset_check && P.scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t base = tile * TILE;
    double lwv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = base + k * TPB + threadIdx.x;
        lwv[k] = -INFINITY;
        if (i >= n)
            continue;
        const double inc = dalpha == 0.0 ? 0.0 : dalpha * llrow[i];
        const double l = (reset ? 0.0 : lw[i]) + inc;
        lw[i] = l;
        lwv[k] = l;
    }
    tile_partial(lwv, part + tile, red);
}

}  // namespace smc
