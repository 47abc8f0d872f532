// smc_gmm_impl.hpp -- (templates over the number of components K) the tempered Bayesian Gaussian-mixture sampler of Section
// 5.2 on gfx950: prior draws, the mixture log-likelihood (and its gradient),
// the three Metropolis blocks (random walk or MALA), and the reweighting by
// the tempering increment.
//
// Per-particle parameters in unconstrained coordinates (rows of the state):
//   mu_j (rows 0..K-1), eta_j = log lambda_j (K..2K-1),
//   z_j = log(omega_j / omega_K) (2K..3K-2), then the cached log-likelihood
//   (row D = 3K-1), log prior (D+1) and, for MALA, the cached likelihood
//   gradient (D+2..2D+1).
//
// The likelihood is the hot loop: l = sum_k lse_j(c_j - lambda_j (y_k -
// mu_j)^2 / 2), c_j = log omega_j + eta_j / 2 - log(2 pi) / 2, i.e. n K
// "mixture terms" per particle, each a subtract, a multiply, a fused
// multiply-add, a max, an exponential and an add, plus one logarithm per
// data point.  A workgroup holds 64 particles (one per lane) and W waves;
// wave w walks its own contiguous chunk of the data with wave-uniform
// (scalar) loads of y, every lane keeps its particle's 3K constants and its
// accumulators in registers, and the W partial sums are combined in wave
// order through LDS.  Nothing here is a dense contraction, so the vector ALU
// (FP64) is the roofline, not the matrix cores.
#include <math.h>

#pragma once

#include "smc_internal.hpp"

namespace smc {

constexpr double kHalfLog2Pi = 0.91893853320467274178032973640562;
constexpr int GMM_MAXW = 8;       // waves per particle tile
constexpr int GMM_RED_GROUP = 4;  // accumulators combined per LDS round
// Where a Metropolis block reads and writes the particles' state: global
// memory both ways (each block its own launch or queue item) or, when one
// workgroup runs a step's blocks in sequence, global -> LDS for the first,
// LDS -> LDS between blocks and LDS -> global for the last.
constexpr int GMM_IO_GLOBAL = 0, GMM_IO_FIRST = 1, GMM_IO_LDS = 2, GMM_IO_LAST = 3;
// doubles of the LDS state copy of one 64-particle tile: D coordinates, the
// log-likelihood, the log prior and, for MALA, the D-gradient
constexpr int gmm_hand_doubles(int K, bool mala)
{
    return (mala ? 2 * (3 * K - 1) + 2 : 3 * K + 1) * WAVE;
}


// log omega_j (j = 0..K-1) from the K-1 logits, reference component K.
template <int K>
__device__ __forceinline__ void log_weights(const double (&phi)[3 * K - 1 > 0 ? 3 * K - 1 : 1],
                                            double (&logw)[K])
{
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
        m = fmax(m, phi[2 * K + j]);
    double s = exp_d(-m);
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
        s += exp_d(phi[2 * K + j] - m);
    const double lse = m + log_d(s);
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
        logw[j] = phi[2 * K + j] - lse;
    logw[K - 1] = -lse;
}

template <int K>
__device__ __forceinline__ double log_prior(const double (&phi)[3 * K - 1 > 0 ? 3 * K - 1 : 1],
                                            const double (&logw)[K], const GmmPrior &pr)
{
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double d = phi[j] - pr.mu_mean;
        a -= d * d * pr.inv_2var;
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        a += pr.shape * phi[K + j] - pr.rate * exp_d(phi[K + j]);
    if (K > 1) {
#pragma unroll
        for (int j = 0; j < K; ++j)
            a += pr.rho * logw[j];
    }
    return a;
}

// gradient of log_prior for the coordinates of one block
template <int K>
__device__ __forceinline__ double log_prior_grad(const double (&phi)[3 * K - 1 > 0 ? 3 * K - 1 : 1],
                                                 const double (&logw)[K], const GmmPrior &pr,
                                                 int q)
{
    if (q < K)
        return -(phi[q] - pr.mu_mean) * (2.0 * pr.inv_2var);
    if (q < 2 * K)
        return pr.shape - pr.rate * exp_d(phi[q]);
    return pr.rho * (1.0 - (double)K * exp_d(logw[q - 2 * K]));
}

// Per-lane mixture likelihood accumulator for one particle (Section 5.2.1):
// log p(y) = log sum_j exp(c_j - (lambda_j / 2) (y - mu_j)^2) with
// c_j = log omega_j + eta_j / 2 - log(2 pi) / 2, summed over the data.
//
// The log-sum-exp of each point runs in base 2: a_j = c_j log2(e) - u_j^2
// with u_j = g_j (y - mu_j) = g_j y - g_j mu_j, g_j = sqrt(lambda_j log2(e)
// / 2), the maximum m of the a_j factored out, s = sum_j 2^(a_j - m) in
// [1, K].  Instead of a logarithm per point, the sums s are multiplied
// together and the product's logarithm is taken every FLUSH points (a
// product of at most 64 factors <= 16 stays below 2^256), so
// log p = ln 2 * sum m + sum log(prod).
//
// Gradient (GRAD): with responsibilities r_j = 2^(a_j - m) / s and
// lambda_j d_j = 2 ln2 g_j u_j, lambda_j d_j^2 / 2 = ln2 u_j^2:
//   d/d mu_j  = sum r_j lambda_j (y - mu_j)        = 2 ln2 g_j sum r_j u_j
//   d/d eta_j = sum r_j (1/2 - lambda_j d_j^2 / 2) = sum r_j / 2 - ln2 sum r_j u_j^2
// accumulated as sum r u (in gmu), sum r u^2 (in geta) and sum r (in gr)
// and converted once in finish().
template <int K, bool GRAD>
struct MixLik {
    static constexpr int FLUSH = 64;
    double g[K], gm[K], c[K];
    double ll;  // after chunk(): sum of log p(y_k) over the chunk
    double m2, lsum, prod;
    double gmu[GRAD ? K : 1], geta[GRAD ? K : 1], gr[GRAD ? K : 1];

    __device__ __forceinline__ void setup(const double (&phi)[3 * K - 1 > 0 ? 3 * K - 1 : 1],
                                          const double (&logw)[K])
    {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            g[j] = sqrt((0.5 * detail::kLog2e) * exp_d(phi[K + j]));
            gm[j] = g[j] * phi[j];
            c[j] = detail::kLog2e * (logw[j] + 0.5 * phi[K + j] - kHalfLog2Pi);
        }
        ll = m2 = lsum = 0.0;
        prod = 1.0;
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                gmu[j] = geta[j] = gr[j] = 0.0;
        }
    }

    // FAST: the terms' 2^x without the clamp that maps x = -inf to 0 (the
    // same value for every finite x; see chunk())
    template <bool FAST = false>
    __device__ __forceinline__ void point(double y)
    {
        double e[K], u[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            u[j] = fma(g[j], y, -gm[j]);
            e[j] = fma(-u[j], u[j], c[j]);
        }
        if constexpr (K == 1) {
            m2 += e[0];
            if (GRAD) {
                gmu[0] += u[0];
                geta[0] = fma(u[0], u[0], geta[0]);
                gr[0] += 1.0;
            }
            return;
        }
        double m = e[0];
#pragma unroll
        for (int j = 1; j < K; ++j)
            m = fmax(m, e[j]);
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            e[j] = FAST ? exp2_nonpos_finite(e[j] - m) : exp2_nonpos(e[j] - m);
            s = j == 0 ? e[0] : s + e[j];
        }
        m2 += m;
        prod *= s;
        if (GRAD) {
            // 1/s for s in [1, K]: hardware estimate and two Newton steps
            double inv = __builtin_amdgcn_rcp(s);
            inv = fma(inv, fma(-s, inv, 1.0), inv);
            inv = fma(inv, fma(-s, inv, 1.0), inv);
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double r = e[j] * inv;
                const double ru = r * u[j];
                gmu[j] += ru;
                geta[j] = fma(ru, u[j], geta[j]);
                gr[j] += r;
            }
        }
    }

    __device__ __forceinline__ void finish()
    {
        ll = fma(detail::kLn2, m2, lsum);
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                gmu[j] *= (2.0 * detail::kLn2) * g[j];
                geta[j] = fma(-detail::kLn2, geta[j], 0.5 * gr[j]);
            }
        }
    }

    // the running sums of a chunk back to their start (the constants of
    // setup() stay)
    __device__ __forceinline__ void reset()
    {
        ll = m2 = lsum = 0.0;
        prod = 1.0;
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                gmu[j] = geta[j] = gr[j] = 0.0;
        }
    }

    // the points [k0, k1) in FLUSH-point segments with wave-uniform loads;
    // in the two-point loop the next pair is loaded one iteration ahead
    template <bool FAST>
    __device__ __forceinline__ void run(const double *__restrict__ y, int64_t k0, int64_t k1)
    {
        int64_t k = k0;
        while (k < k1) {
            const int64_t kend = min(k + FLUSH, k1);
            if (K <= 8) {  // two points per iteration while registers allow
                if (k + 2 <= kend) {
                    double y0 = y[k], y1 = y[k + 1];
                    if constexpr (FAST && !GRAD) {
                        // unrolled once more: the prefetched pair alternates
                        // between two register pairs instead of being moved
#pragma unroll 2
                        for (; k + 4 <= kend; k += 2) {
                            const double n0 = y[k + 2], n1 = y[k + 3];
                            point<FAST>(y0);
                            point<FAST>(y1);
                            y0 = n0;
                            y1 = n1;
                        }
                    } else {
                        for (; k + 4 <= kend; k += 2) {
                            const double n0 = y[k + 2], n1 = y[k + 3];
                            point<FAST>(y0);
                            point<FAST>(y1);
                            y0 = n0;
                            y1 = n1;
                        }
                    }
                    point<FAST>(y0);
                    point<FAST>(y1);
                    k += 2;
                }
            }
            for (; k < kend; ++k)
                point<FAST>(y[k]);
            lsum += log_d(prod);
            prod = 1.0;
        }
        finish();
    }

    // accumulate a contiguous chunk of the data: first with the terms' 2^x
    // unclamped; a non-finite term makes the log-likelihood NaN, and then the
    // chunk is summed again with the clamp, so the results are those of the
    // clamped form for every input
    __device__ __forceinline__ void chunk(const double *__restrict__ y, int64_t k0, int64_t k1)
    {
        if constexpr (K > 1) {
            run<true>(y, k0, k1);
            if (!(ll == ll)) {
                reset();
                run<false>(y, k0, k1);
            }
        } else {
            run<false>(y, k0, k1);
        }
    }

    static constexpr int NACC = GRAD ? 1 + 3 * K : 1;
    __device__ __forceinline__ double &acc(int q)
    {
        if (q == 0)
            return ll;
        if (q <= K)
            return gmu[GRAD ? q - 1 : 0];
        if (q <= 2 * K)
            return geta[GRAD ? q - 1 - K : 0];
        return gr[GRAD ? q - 1 - 2 * K : 0];
    }
};

// Combines the accumulators of the W waves in wave order; wave 0 ends with
// the totals.  `red` holds GMM_RED_GROUP * GMM_MAXW * 64 doubles.
template <int K, bool GRAD>
__device__ __forceinline__ void combine_waves(MixLik<K, GRAD> &L, int W, double *red)
{
    constexpr int NACC = MixLik<K, GRAD>::NACC;
    const int w = wave_id(), lane = lane_id();
    for (int q0 = 0; q0 < NACC; q0 += GMM_RED_GROUP) {
        __syncthreads();
        if (w > 0) {
#pragma unroll
            for (int g = 0; g < GMM_RED_GROUP; ++g)
                if (q0 + g < NACC)
                    red[(g * GMM_MAXW + w) * WAVE + lane] = L.acc(q0 + g);
        }
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int g = 0; g < GMM_RED_GROUP; ++g)
                if (q0 + g < NACC) {
                    double a = L.acc(q0 + g);
                    for (int v = 1; v < W; ++v)
                        a += red[(g * GMM_MAXW + v) * WAVE + lane];
                    L.acc(q0 + g) = a;
                }
        }
    }
}

// Wave w's share [k0, k1) of the n data points (uniform across the wave).
__device__ __forceinline__ void data_chunk(int64_t nd, int W, int64_t *k0, int64_t *k1)
{
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    const int64_t per = (nd + W - 1) / W;
    *k0 = min((int64_t)w * per, nd);
    *k1 = min(*k0 + per, nd);
}

// z-gradient from the accumulated responsibilities: sum_k (r_kj - omega_j)
template <int K>
__device__ __forceinline__ double z_grad(double gr_j, double logw_j, int64_t nd)
{
    return gr_j - (double)nd * exp_d(logw_j);
}

// ---------------------------------------------------------------------------
// Initialisation from the prior (Algorithm "gmm"): mu_j = xi + sd n_j
// (normals: call j/2), lambda_j = G_j / b with G_j ~ Gamma(a) (calls from
// 64 + 64 j), omega = H / sum H with H_j ~ Gamma(rho) (calls from
// 64 + 1024 + 64 j); then log prior and log-likelihood (and its gradient for
// MALA); log-weights 0.
// ---------------------------------------------------------------------------
template <int K, bool GRAD>
__device__ __forceinline__ void gmm_init_tile(const Prob &P, int W, int64_t tile)
{
    constexpr int D = 3 * K - 1;
    __shared__ double red[GMM_RED_GROUP * GMM_MAXW * WAVE];
    double *__restrict__ st = (double *)P.state[0];
    double *__restrict__ lw = P.lw;
    const int64_t n = P.n, nd = P.n_data;
    const double *__restrict__ y = P.data;
    const Key key = P.key;
    const uint32_t p = P.problem_id;
    const GmmPrior pr = P.prior;
    const double mu_sd = P.mu_sd;
    int32_t *__restrict__ counters = P.counters;
    const int64_t i = tile * WAVE + lane_id();
    const bool valid = i < n;
    const uint32_t ii = (uint32_t)(valid ? i : 0);
    double phi[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < K; j += 2) {
        const double2 z = normal2(draw(key, ii, 0, TAG_INIT, (uint32_t)(j / 2), p));
        phi[j] = pr.mu_mean + mu_sd * z.x;
        if (j + 1 < K)
            phi[j + 1] = pr.mu_mean + mu_sd * z.y;
    }
    int fail = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double G = gamma_draw(key, ii, 0, TAG_INIT, (uint32_t)(64 + 64 * j), p, pr.shape,
                                    &fail);
        phi[K + j] = log_d(G / pr.rate);
    }
    double H[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        H[j] = gamma_draw(key, ii, 0, TAG_INIT, (uint32_t)(64 + 64 * 16 + 64 * j), p, pr.rho,
                          &fail);
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
        phi[2 * K + j] = log_d(H[j]) - log_d(H[K - 1]);
    double logw[K];
    log_weights<K>(phi, logw);
    MixLik<K, GRAD> L;
    L.setup(phi, logw);
    int64_t k0, k1;
    data_chunk(nd, W, &k0, &k1);
    L.chunk(y, k0, k1);
    combine_waves<K, GRAD>(L, W, red);
    if (wave_id() == 0 && valid) {
#pragma unroll
        for (int q = 0; q < D; ++q)
            st[(int64_t)q * n + i] = phi[q];
        st[(int64_t)D * n + i] = L.ll;
        st[(int64_t)(D + 1) * n + i] = log_prior<K>(phi, logw, pr);
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                st[(int64_t)(D + 2 + j) * n + i] = L.gmu[j];
                st[(int64_t)(D + 2 + K + j) * n + i] = L.geta[j];
                if (j < K - 1)
                    st[(int64_t)(D + 2 + 2 * K + j) * n + i] = z_grad<K>(L.gr[j], logw[j], nd);
            }
        }
        lw[i] = 0.0;
        if (fail)
            atomicOr(&counters[CNT_ERR], SMC_DEVERR_GAMMA);
    }
}

template <int K, bool GRAD>
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_init_kernel(Prob P, int W)
{
    gmm_init_tile<K, GRAD>(P, W, blockIdx.x);
}

template <int K, bool GRAD>
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_init_batch_kernel(
    const Prob *__restrict__ probs, const int2 *__restrict__ map, int W)
{
    const int2 pm = map[blockIdx.x];
    gmm_init_tile<K, GRAD>(probs[pm.x], W, pm.y);
}

// ---------------------------------------------------------------------------
// One Metropolis block of every particle at tempering alpha (the three-block
// kernel of Section 5.2.1).  Random walk: phi'_b = phi_b + s n.  MALA:
// phi'_b = phi_b + s^2/2 g + s n, g the block gradient of prior + alpha x
// likelihood, with both proposal densities in the ratio.  Accept iff
// log u <= log r.  With `full` every row is written to the ping-pong
// partner (the first block after a resample call), the particle read through
// the pending ancestors when the resample happened; otherwise the accepted
// rows are updated in place.  Accepted proposals are counted into
// history[step][ACC0 + block] (integer-valued, so the order of the additions
// does not matter).
// ---------------------------------------------------------------------------
// The proposal of particle i for one block: loads phi, draws the normals,
// adds the drift (MALA).  Deterministic, so it is rebuilt after the data
// loop instead of being kept in registers across it.  All array indices are
// compile-time (the block's coordinates are selected by uniform branches),
// so nothing is spilled to scratch.  fwd = sum over the block of
// (phi' - phi - drift)^2, the forward proposal term of MALA.
template <int K, bool MALA>
struct Proposal {
    static constexpr int D = 3 * K - 1;
    double phi[D > 0 ? D : 1];
    double prop[D > 0 ? D : 1];
    double logw0[K];
    double fwd;

    __device__ __forceinline__ void build(const double *__restrict__ src, int64_t n, int64_t si,
                                          uint32_t ii, Key key, uint32_t t, uint32_t p, int block,
                                          int sweep, double alpha, double scale,
                                          const GmmPrior &pr)
    {
        const int off = block * K;
        const int dim = block == 2 ? K - 1 : K;
#pragma unroll
        for (int q = 0; q < D; ++q)
            phi[q] = src[(int64_t)q * n + si];
        log_weights<K>(phi, logw0);
        const uint32_t tag = TAG_MH_MU + (uint32_t)block;
        const double h2 = scale * scale;
        fwd = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q)
            prop[q] = phi[q];
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int mm = q - off;
            if (mm >= 0 && mm < dim && (mm & 1) == 0) {
                const double2 z =
                    normal2(draw(key, ii, t, tag, (uint32_t)(64 * sweep + mm / 2), p));
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (q + h < D && mm + h < dim) {
                        const double xi = h == 0 ? z.x : z.y;
                        double dr = 0.0;
                        if (MALA) {
                            double g = log_prior_grad<K>(phi, logw0, pr, q + h);
                            if (alpha != 0.0)
                                g += alpha * src[(int64_t)(D + 2 + q + h) * n + si];
                            dr = 0.5 * h2 * g;
                        }
                        const double v = phi[q + h] + dr + scale * xi;
                        prop[q + h] = v;
                        const double a = v - phi[q + h] - dr;
                        fwd += a * a;
                    }
                }
            }
        }
    }
};

// Values of the epilogue that do not depend on the likelihood, computed
// before the data loop by the last wave and kept in LDS (one column per
// lane) until wave 0 takes the decision: the proposal's log prior, the log of
// the accept uniform, the proposed block coordinates and, for MALA, the
// forward proposal term, the prior gradient at the proposal (block
// coordinates) and the proposed mixture weights omega'_j (the z-gradient
// subtracts n omega'_j).
template <int K, bool MALA>
struct BlockStash {
    static constexpr int LPP = 0, LOGU = 1, FWD = 2, PROP = 3, GP = 3 + K, ZC = 3 + 2 * K;
    static constexpr int ROWS = MALA ? 3 + 3 * K - 1 : 3 + K;
};

// LDS of one Metropolis block: the wave-combine buffer and the stash.
constexpr int GMM_RED_DOUBLES = GMM_RED_GROUP * GMM_MAXW * WAVE;
template <int K, bool MALA>
constexpr int gmm_stash_doubles() { return BlockStash<K, MALA>::ROWS * WAVE; }

// `red` (GMM_RED_DOUBLES), `stash` (gmm_stash_doubles<K, MALA>()) and, for
// the LDS hand-off modes `io`, `hand` (gmm_hand_doubles(K, MALA)) are the
// caller's LDS.  With GMM_IO_GLOBAL the block reads `src` and writes `dst`
// (every row when `full`, else the accepted rows in place).
template <int K, bool MALA>
__device__ __forceinline__ void gmm_block_tile(const Prob &P, const double *__restrict__ src,
                                               double *__restrict__ dst, int full, int W,
                                               int64_t tile, uint32_t t, int block, int sweep,
                                               double alpha, double scale, int32_t step,
                                               double *red, double *stash, int io = GMM_IO_GLOBAL,
                                               double *hand = nullptr)
{
    constexpr int D = 3 * K - 1;
    using S = BlockStash<K, MALA>;
    const bool in_lds = io == GMM_IO_LDS || io == GMM_IO_LAST;
    const bool out_lds = io == GMM_IO_FIRST || io == GMM_IO_LDS;
    const bool out_all = full || io != GMM_IO_GLOBAL;
    const int32_t *__restrict__ anc = P.anc;
    const int64_t n = P.n, nd = P.n_data;
    const double *__restrict__ y = P.data;
    const Key key = P.key;
    const uint32_t p = P.problem_id;
    const GmmPrior pr = P.prior;
    double *__restrict__ hist = P.hist;
    const int64_t hist_len = P.hist_len;
    const bool gather = full && !in_lds && P.scalars[SMC_S_RESAMPLED] != 0.0;
    const int lane = lane_id();
    const int64_t i = tile * WAVE + lane;
    const bool valid = i < n;
    // the state is read from column si of rows of length sn (global: the
    // particle or its ancestor; LDS: the lane) and written to column wi of
    // rows of length wn
    const int64_t si = in_lds ? lane : (valid ? (gather ? (int64_t)anc[i] : i) : 0);
    const int64_t sn = in_lds ? WAVE : n;
    const double *__restrict__ rs = in_lds ? hand : src;
    double *__restrict__ ws = out_lds ? hand : dst;
    const int64_t wi = out_lds ? lane : i;
    const int64_t wn = out_lds ? WAVE : n;
    const uint32_t ii = (uint32_t)(valid ? i : 0);
    const int off = block * K;
    const int dim = block == 2 ? K - 1 : K;
    const double h2 = scale * scale;
    MixLik<K, MALA> L;
    {
        Proposal<K, MALA> Q;
        Q.build(rs, sn, si, ii, key, t, p, block, sweep, alpha, scale, pr);
        double logw[K];
        log_weights<K>(Q.prop, logw);
        L.setup(Q.prop, logw);
        if (__builtin_amdgcn_readfirstlane(wave_id()) == W - 1) {
            stash[S::LPP * WAVE + lane] = log_prior<K>(Q.prop, logw, pr);
            const uint4 wa = draw(key, ii, t, TAG_MH_ACCEPT, (uint32_t)(4 * sweep + block), p);
            stash[S::LOGU * WAVE + lane] = log_d(u53(wa.x, wa.y));
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int mm = q - off;
                if (mm >= 0 && mm < dim) {
                    stash[(S::PROP + mm) * WAVE + lane] = Q.prop[q];
                    if (MALA)
                        stash[(S::GP + mm) * WAVE + lane] = log_prior_grad<K>(Q.prop, logw, pr, q);
                }
            }
            if (MALA) {
                stash[S::FWD * WAVE + lane] = Q.fwd;
#pragma unroll
                for (int j = 0; j < K - 1; ++j)
                    stash[(S::ZC + j) * WAVE + lane] = exp_d(logw[j]);
            }
        }
    }
    int64_t k0, k1;
    data_chunk(nd, W, &k0, &k1);
    L.chunk(y, k0, k1);
    double ll0 = 0.0, lp0 = 0.0;
    if (wave_id() == 0) {
        ll0 = rs[(int64_t)D * sn + si];
        lp0 = rs[(int64_t)(D + 1) * sn + si];
    }
    combine_waves<K, MALA>(L, W, red);
    if (wave_id() != 0)
        return;
    double phi[D > 0 ? D : 1];
#pragma unroll
    for (int q = 0; q < D; ++q)
        phi[q] = rs[(int64_t)q * sn + si];
    const double lpp = stash[S::LPP * WAVE + lane];
    const double cur = alpha == 0.0 ? lp0 : lp0 + alpha * ll0;
    double logr = (alpha == 0.0 ? lpp : lpp + alpha * L.ll) - cur;
    double gnew[MALA ? D : 1];
    if (MALA) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            gnew[j] = L.gmu[j];
            gnew[K + j] = L.geta[j];
            if (j < K - 1)
                gnew[2 * K + j] = L.gr[j] - (double)nd * stash[(S::ZC + j) * WAVE + lane];
        }
        double bwd = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int mm = q - off;
            if (mm >= 0 && mm < dim) {
                double g2 = stash[(S::GP + mm) * WAVE + lane];
                if (alpha != 0.0)
                    g2 += alpha * gnew[q];
                const double b = phi[q] - stash[(S::PROP + mm) * WAVE + lane] - 0.5 * h2 * g2;
                bwd += b * b;
            }
        }
        logr += (stash[S::FWD * WAVE + lane] - bwd) / (2.0 * h2);
    }
    const bool acc = valid && stash[S::LOGU * WAVE + lane] <= logr;
    if (valid || out_lds) {
        if (out_all) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int mm = q - off;
                const bool inb = mm >= 0 && mm < dim;
                ws[(int64_t)q * wn + wi] =
                    (acc && inb) ? stash[(S::PROP + (inb ? mm : 0)) * WAVE + lane] : phi[q];
            }
            ws[(int64_t)D * wn + wi] = acc ? L.ll : ll0;
            ws[(int64_t)(D + 1) * wn + wi] = acc ? lpp : lp0;
            if (MALA) {
#pragma unroll
                for (int q = 0; q < D; ++q)
                    ws[(int64_t)(D + 2 + q) * wn + wi] =
                        acc ? gnew[q] : rs[(int64_t)(D + 2 + q) * sn + si];
            }
        } else if (acc) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const int mm = q - off;
                if (mm >= 0 && mm < dim)
                    ws[(int64_t)q * wn + wi] = stash[(S::PROP + mm) * WAVE + lane];
            }
            ws[(int64_t)D * wn + wi] = L.ll;
            ws[(int64_t)(D + 1) * wn + wi] = lpp;
            if (MALA) {
#pragma unroll
                for (int q = 0; q < D; ++q)
                    ws[(int64_t)(D + 2 + q) * wn + wi] = gnew[q];
            }
        }
    }
    // count accepted proposals of this wave
    const unsigned long long bal = __ballot(acc);
    if (lane == 0 && hist && step >= 0 && step < hist_len && bal)
        atomicAdd(&hist[(int64_t)step * SMC_HIST_COLS + SMC_H_ACC0 + block],
                  (double)__popcll(bal));
}

// All Metropolis blocks of a step (every sweep) in one launch: the tile's
// workgroup runs the blocks one after the other.  The first block reads
// `src` (through the ancestors when the step resampled and `full` is set)
// and leaves the tile's state in LDS; each later block reads the state the
// previous block's wave 0 left there (visible to the workgroup after the
// barrier), and the last one writes the whole state to `dst`.
template <int K, bool MALA>
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_step_kernel(
    Prob P, const double *__restrict__ src, double *__restrict__ dst, int full, int W, uint32_t t,
    int sweeps, double alpha, double s0, double s1, double s2, int32_t step)
{
    __shared__ double red[GMM_RED_DOUBLES];
    __shared__ double stash[gmm_stash_doubles<K, MALA>()];
    __shared__ double hand[gmm_hand_doubles(K, MALA)];
    const int nb = K == 1 ? 2 : 3;
    for (int sw = 0; sw < sweeps; ++sw)
        for (int b = 0; b < nb; ++b) {
            const bool first = sw == 0 && b == 0;
            const bool last = sw == sweeps - 1 && b == nb - 1;
            if (!first)
                __syncthreads();
            gmm_block_tile<K, MALA>(P, src, dst, first ? full : 0, W, blockIdx.x, t, b, sw, alpha,
                                    b == 0 ? s0 : (b == 1 ? s1 : s2), step, red, stash,
                                    first ? GMM_IO_FIRST : (last ? GMM_IO_LAST : GMM_IO_LDS),
                                    hand);
        }
}

// ---------------------------------------------------------------------------
// Log-likelihood (and gradient) for separate parameter arrays (the adjoint
// entry point).
// ---------------------------------------------------------------------------
template <int K, bool GRAD>
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_loglik_kernel(
    const double *__restrict__ mu, const double *__restrict__ eta, const double *__restrict__ z,
    int64_t n, const double *__restrict__ y, int64_t nd, int W, double *__restrict__ ll,
    double *__restrict__ grad)
{
    constexpr int D = 3 * K - 1;
    __shared__ double red[GMM_RED_GROUP * GMM_MAXW * WAVE];
    const int64_t i = (int64_t)blockIdx.x * WAVE + lane_id();
    const bool valid = i < n;
    const int64_t si = valid ? i : 0;
    double phi[D > 0 ? D : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        phi[j] = mu[(int64_t)j * n + si];
        phi[K + j] = eta[(int64_t)j * n + si];
        if (j < K - 1)
            phi[2 * K + j] = z[(int64_t)j * n + si];
    }
    double logw[K];
    log_weights<K>(phi, logw);
    MixLik<K, GRAD> L;
    L.setup(phi, logw);
    int64_t k0, k1;
    data_chunk(nd, W, &k0, &k1);
    L.chunk(y, k0, k1);
    combine_waves<K, GRAD>(L, W, red);
    if (wave_id() == 0 && valid) {
        ll[i] = L.ll;
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                grad[(int64_t)j * n + i] = L.gmu[j];
                grad[(int64_t)(K + j) * n + i] = L.geta[j];
                if (j < K - 1)
                    grad[(int64_t)(2 * K + j) * n + i] = z_grad<K>(L.gr[j], logw[j], nd);
            }
        }
    }
}

// Host launchers of the K-templated kernels; explicitly instantiated in the
// smc_gmm_k*.hip translation units (compiled in parallel).
int gmm_waves(int64_t n, int64_t nd);

template <int K>
struct GmmK {
    static hipError_t init(Ctx &c, int W);
    static hipError_t step(Ctx &c, int W, int32_t step, int sweeps, double alpha,
                           const double (&scale)[3], bool gather_check);
    static hipError_t loglik(const double *mu, const double *eta, const double *z, int64_t n,
                             const double *y, int64_t nd, double *ll, double *grad, hipStream_t s);
    static hipError_t init_batch(const Prob *probs, const int2 *map, int64_t tiles, int W,
                                 bool mala, hipStream_t s);
};

template <int K>
hipError_t GmmK<K>::init(Ctx &c, int W)
{
    const dim3 grid((unsigned)ceil_div(c.n, WAVE)), block((unsigned)(W * WAVE));
    const Key key = make_key(c.cfg.seed);
    const Prob P = make_prob(c);
    (void)key;
    if (c.cfg.move_kind == SMC_MOVE_MALA)
        hipLaunchKernelGGL((gmm_init_kernel<K, true>), grid, block, 0, c.stream, P, W);
    else
        hipLaunchKernelGGL((gmm_init_kernel<K, false>), grid, block, 0, c.stream, P, W);
    return hipGetLastError();
}

template <int K>
hipError_t GmmK<K>::step(Ctx &c, int W, int32_t step, int sweeps, double alpha,
                         const double (&scale)[3], bool gather_check)
{
    const dim3 grid((unsigned)ceil_div(c.n, WAVE)), blk((unsigned)(W * WAVE));
    const double *src = (const double *)c.state_ptr();
    double *dst = gather_check ? (double *)c.other_ptr() : (double *)c.state_ptr();
    const Prob P = make_prob(c);
    hipEvent_t e0, e1;
    const bool timed = c.prof_take(&e0, &e1);
#define SMC_STEP_ARGS                                                                             \
    P, src, dst, (int)gather_check, W, (uint32_t)step, sweeps, alpha, scale[0], scale[1],         \
        scale[2], step
    if (c.cfg.move_kind == SMC_MOVE_MALA) {
        if (timed)
            hipExtLaunchKernelGGL((gmm_step_kernel<K, true>), grid, blk, 0, c.stream, e0, e1, 0,
                                  SMC_STEP_ARGS);
        else
            hipLaunchKernelGGL((gmm_step_kernel<K, true>), grid, blk, 0, c.stream, SMC_STEP_ARGS);
    } else {
        if (timed)
            hipExtLaunchKernelGGL((gmm_step_kernel<K, false>), grid, blk, 0, c.stream, e0, e1, 0,
                                  SMC_STEP_ARGS);
        else
            hipLaunchKernelGGL((gmm_step_kernel<K, false>), grid, blk, 0, c.stream,
                               SMC_STEP_ARGS);
    }
#undef SMC_STEP_ARGS
    return hipGetLastError();
}

template <int K>
hipError_t GmmK<K>::loglik(const double *mu, const double *eta, const double *z, int64_t n,
                                  const double *y, int64_t nd, double *ll, double *grad,
                                  hipStream_t s)
{
    const int W = gmm_waves(n, nd);
    const dim3 grid((unsigned)ceil_div(n, WAVE)), blk((unsigned)(W * WAVE));
    if (grad)
        hipLaunchKernelGGL((gmm_loglik_kernel<K, true>), grid, blk, 0, s, mu, eta, z, n, y, nd,
                           W, ll, grad);
    else
        hipLaunchKernelGGL((gmm_loglik_kernel<K, false>), grid, blk, 0, s, mu, eta, z, n, y, nd,
                           W, ll, grad);
    return hipGetLastError();
}

template <int K>
hipError_t GmmK<K>::init_batch(const Prob *probs, const int2 *map, int64_t tiles, int W,
                                      bool mala, hipStream_t s)
{
    const dim3 grid((unsigned)tiles), blk((unsigned)(W * WAVE));
    if (mala)
        hipLaunchKernelGGL((gmm_init_batch_kernel<K, true>), grid, blk, 0, s, probs, map, W);
    else
        hipLaunchKernelGGL((gmm_init_batch_kernel<K, false>), grid, blk, 0, s, probs, map, W);
    return hipGetLastError();
}


}  // namespace smc
