// smc_gmm.hip -- the tempered Bayesian Gaussian-mixture sampler of Section
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

#include "smc_internal.hpp"

namespace smc {

constexpr double kHalfLog2Pi = 0.91893853320467274178032973640562;
constexpr int GMM_MAXW = 8;       // waves per particle tile
constexpr int GMM_RED_GROUP = 4;  // accumulators combined per LDS round

struct GmmPrior {
    double mu_mean, inv_2var, shape, rate, rho;
};

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

// Per-lane mixture likelihood accumulator for one particle.
template <int K, bool GRAD>
struct MixLik {
    double mu[K], hl[K], c[K];
    double ll;
    double gmu[GRAD ? K : 1], geta[GRAD ? K : 1], gr[GRAD ? K : 1];

    __device__ __forceinline__ void setup(const double (&phi)[3 * K - 1 > 0 ? 3 * K - 1 : 1],
                                          const double (&logw)[K])
    {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            mu[j] = phi[j];
            hl[j] = 0.5 * exp_d(phi[K + j]);
            c[j] = logw[j] + 0.5 * phi[K + j] - kHalfLog2Pi;
        }
        ll = 0.0;
        if (GRAD) {
#pragma unroll
            for (int j = 0; j < K; ++j)
                gmu[j] = geta[j] = gr[j] = 0.0;
        }
    }

    __device__ __forceinline__ void point(double y)
    {
        double e[K], d[K];
        double m = -INFINITY;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            d[j] = y - mu[j];
            e[j] = fma(-hl[j] * d[j], d[j], c[j]);
            m = fmax(m, e[j]);
        }
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            e[j] = exp_d(e[j] - m);
            s += e[j];
        }
        ll += m + log_d(s);
        if (GRAD) {
            const double inv = 1.0 / s;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const double r = e[j] * inv;
                const double rh = r * hl[j];
                gmu[j] = fma(2.0 * rh, d[j], gmu[j]);
                geta[j] = fma(-rh * d[j], d[j], fma(0.5, r, geta[j]));
                gr[j] += r;
            }
        }
    }

    // accumulate a contiguous chunk of the data with wave-uniform loads
    __device__ __forceinline__ void chunk(const double *__restrict__ y, int64_t k0, int64_t k1)
    {
        int64_t k = k0;
        for (; k + 2 <= k1; k += 2) {
            const double y0 = y[k], y1 = y[k + 1];
            point(y0);
            point(y1);
        }
        if (k < k1)
            point(y[k]);
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
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_init_kernel(
    double *__restrict__ st, double *__restrict__ lw, int64_t n, const double *__restrict__ y,
    int64_t nd, int W, Key key, uint32_t p, GmmPrior pr, double mu_sd,
    int32_t *__restrict__ counters)
{
    constexpr int D = 3 * K - 1;
    __shared__ double red[GMM_RED_GROUP * GMM_MAXW * WAVE];
    const int64_t i = (int64_t)blockIdx.x * WAVE + lane_id();
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

// Tile partials of all-zero log-weights: m = 0, s1 = s2 = particles in tile.
__global__ void const_partials_kernel(TilePartial *__restrict__ part, int64_t ntiles, int64_t n)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < ntiles) {
        const double len = (double)min((int64_t)TILE, n - b * TILE);
        part[b] = TilePartial{0.0, len, len, 0.0};
    }
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

template <int K, bool MALA>
__global__ __launch_bounds__(GMM_MAXW *WAVE) void gmm_block_kernel(
    const double *__restrict__ src, double *__restrict__ dst, const int32_t *__restrict__ anc,
    const double *__restrict__ scalars, int full, int64_t n, const double *__restrict__ y,
    int64_t nd, int W, Key key, uint32_t t, uint32_t p, int block, int sweep, double alpha,
    double scale, GmmPrior pr, double *__restrict__ hist, int64_t hist_len, int32_t step)
{
    constexpr int D = 3 * K - 1;
    __shared__ double red[GMM_RED_GROUP * GMM_MAXW * WAVE];
    const bool gather = full && scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t i = (int64_t)blockIdx.x * WAVE + lane_id();
    const bool valid = i < n;
    const int64_t si = valid ? (gather ? (int64_t)anc[i] : i) : 0;
    const uint32_t ii = (uint32_t)(valid ? i : 0);
    const int off = block * K;
    const int dim = block == 2 ? K - 1 : K;
    MixLik<K, MALA> L;
    {
        Proposal<K, MALA> P;
        P.build(src, n, si, ii, key, t, p, block, sweep, alpha, scale, pr);
        double logw[K];
        log_weights<K>(P.prop, logw);
        L.setup(P.prop, logw);
    }
    int64_t k0, k1;
    data_chunk(nd, W, &k0, &k1);
    L.chunk(y, k0, k1);
    combine_waves<K, MALA>(L, W, red);
    if (wave_id() != 0)
        return;
    Proposal<K, MALA> P;
    P.build(src, n, si, ii, key, t, p, block, sweep, alpha, scale, pr);
    double logw[K];
    log_weights<K>(P.prop, logw);
    const double ll0 = src[(int64_t)D * n + si];
    const double lp0 = src[(int64_t)(D + 1) * n + si];
    const double lpp = log_prior<K>(P.prop, logw, pr);
    const double cur = alpha == 0.0 ? lp0 : lp0 + alpha * ll0;
    double logr = (alpha == 0.0 ? lpp : lpp + alpha * L.ll) - cur;
    double gnew[MALA ? D : 1];
    if (MALA) {
        const double h2 = scale * scale;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            gnew[j] = L.gmu[j];
            gnew[K + j] = L.geta[j];
            if (j < K - 1)
                gnew[2 * K + j] = z_grad<K>(L.gr[j], logw[j], nd);
        }
        double bwd = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const int mm = q - off;
            if (mm >= 0 && mm < dim) {
                double g2 = log_prior_grad<K>(P.prop, logw, pr, q);
                if (alpha != 0.0)
                    g2 += alpha * gnew[q];
                const double b = P.phi[q] - P.prop[q] - 0.5 * h2 * g2;
                bwd += b * b;
            }
        }
        logr += (P.fwd - bwd) / (2.0 * h2);
    }
    const uint4 wa = draw(key, ii, t, TAG_MH_ACCEPT, (uint32_t)(4 * sweep + block), p);
    const bool acc = valid && log_d(u53(wa.x, wa.y)) <= logr;
    if (valid) {
        if (full) {
#pragma unroll
            for (int q = 0; q < D; ++q)
                dst[(int64_t)q * n + i] = acc ? P.prop[q] : P.phi[q];
            dst[(int64_t)D * n + i] = acc ? L.ll : ll0;
            dst[(int64_t)(D + 1) * n + i] = acc ? lpp : lp0;
            if (MALA) {
#pragma unroll
                for (int q = 0; q < D; ++q)
                    dst[(int64_t)(D + 2 + q) * n + i] =
                        acc ? gnew[q] : src[(int64_t)(D + 2 + q) * n + si];
            }
        } else if (acc) {
#pragma unroll
            for (int q = 0; q < D; ++q)
                if (q >= off && q < off + dim)
                    dst[(int64_t)q * n + i] = P.prop[q];
            dst[(int64_t)D * n + i] = L.ll;
            dst[(int64_t)(D + 1) * n + i] = lpp;
            if (MALA) {
#pragma unroll
                for (int q = 0; q < D; ++q)
                    dst[(int64_t)(D + 2 + q) * n + i] = gnew[q];
            }
        }
    }
    // count accepted proposals of this wave
    const unsigned long long bal = __ballot(acc);
    if (lane_id() == 0 && hist && step >= 0 && step < hist_len && bal)
        atomicAdd(&hist[(int64_t)step * SMC_HIST_COLS + SMC_H_ACC0 + block],
                  (double)__popcll(bal));
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

// ---------------------------------------------------------------------------
// Reweighting of Algorithm "gmm": lw <- (reset ? 0 : lw) + dalpha * l, with
// dalpha == 0 adding exactly 0; per-tile partials for the normalisation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TPB) void gmm_reweight_kernel(
    double *__restrict__ lw, const double *__restrict__ llrow, const double *__restrict__ scalars,
    int reset_check, double dalpha, int64_t n, TilePartial *__restrict__ part)
{
    __shared__ double red[NWAVES];
    const bool reset = reset_check && scalars[SMC_S_RESAMPLED] != 0.0;
    const int64_t base = (int64_t)blockIdx.x * TILE;
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
    tile_partial(lwv, part + blockIdx.x, red);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
static GmmPrior make_prior(const smc_config &c)
{
    return GmmPrior{c.prior_mu_mean, 1.0 / (2.0 * c.prior_mu_sd * c.prior_mu_sd),
                    c.prior_gamma_shape, c.prior_gamma_rate, c.prior_dir_rho};
}

// Waves per 64-particle tile: enough waves overall to fill the GPU, at most
// GMM_MAXW, and no more than the data can feed (>= 32 points per wave).
int gmm_waves(int64_t n, int64_t nd)
{
    const int64_t tiles = ceil_div(n, WAVE);
    int W = 1;
    while (W < GMM_MAXW && tiles * W < 8192 && nd >= (int64_t)(2 * W) * 32)
        W *= 2;
    return W;
}

template <int K>
static hipError_t dispatch_init(Ctx &c, int W)
{
    const dim3 grid((unsigned)ceil_div(c.n, WAVE)), block((unsigned)(W * WAVE));
    const Key key = make_key(c.cfg.seed);
    if (c.cfg.move_kind == SMC_MOVE_MALA)
        hipLaunchKernelGGL((gmm_init_kernel<K, true>), grid, block, 0, c.stream,
                           (double *)c.state_ptr(), c.buf.log_weight, c.n, c.buf.data,
                           c.cfg.n_data, W, key, c.cfg.problem_id, make_prior(c.cfg),
                           c.cfg.prior_mu_sd, c.counters());
    else
        hipLaunchKernelGGL((gmm_init_kernel<K, false>), grid, block, 0, c.stream,
                           (double *)c.state_ptr(), c.buf.log_weight, c.n, c.buf.data,
                           c.cfg.n_data, W, key, c.cfg.problem_id, make_prior(c.cfg),
                           c.cfg.prior_mu_sd, c.counters());
    return hipGetLastError();
}

template <int K>
static hipError_t dispatch_block(Ctx &c, int W, int32_t step, int block, int sweep, double alpha,
                                 double scale, bool gather_check)
{
    const dim3 grid((unsigned)ceil_div(c.n, WAVE)), blk((unsigned)(W * WAVE));
    const Key key = make_key(c.cfg.seed);
    const double *src = (const double *)c.state_ptr();
    double *dst = gather_check ? (double *)c.other_ptr() : (double *)c.state_ptr();
    if (c.cfg.move_kind == SMC_MOVE_MALA)
        hipLaunchKernelGGL((gmm_block_kernel<K, true>), grid, blk, 0, c.stream, src, dst,
                           c.buf.ancestors, c.buf.scalars, (int)gather_check, c.n, c.buf.data,
                           c.cfg.n_data, W, key, (uint32_t)step, c.cfg.problem_id, block, sweep,
                           alpha, scale, make_prior(c.cfg), c.buf.history, c.buf.history_len,
                           step);
    else
        hipLaunchKernelGGL((gmm_block_kernel<K, false>), grid, blk, 0, c.stream, src, dst,
                           c.buf.ancestors, c.buf.scalars, (int)gather_check, c.n, c.buf.data,
                           c.cfg.n_data, W, key, (uint32_t)step, c.cfg.problem_id, block, sweep,
                           alpha, scale, make_prior(c.cfg), c.buf.history, c.buf.history_len,
                           step);
    return hipGetLastError();
}

template <int K>
static hipError_t dispatch_loglik(const double *mu, const double *eta, const double *z, int64_t n,
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

#define SMC_K_SWITCH(K_, CALL)                                                                   \
    switch (K_) {                                                                                \
    case 1: return CALL(1);                                                                      \
    case 2: return CALL(2);                                                                      \
    case 3: return CALL(3);                                                                      \
    case 4: return CALL(4);                                                                      \
    case 5: return CALL(5);                                                                      \
    case 6: return CALL(6);                                                                      \
    case 7: return CALL(7);                                                                      \
    case 8: return CALL(8);                                                                      \
    case 9: return CALL(9);                                                                      \
    case 10: return CALL(10);                                                                    \
    case 11: return CALL(11);                                                                    \
    case 12: return CALL(12);                                                                    \
    case 13: return CALL(13);                                                                    \
    case 14: return CALL(14);                                                                    \
    case 15: return CALL(15);                                                                    \
    case 16: return CALL(16);                                                                    \
    default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_gmm_init(Ctx &c)
{
    const int W = gmm_waves(c.n, c.cfg.n_data);
#define CALL_INIT(k) dispatch_init<k>(c, W)
    hipError_t e;
    {
        auto f = [&]() -> hipError_t { SMC_K_SWITCH(c.cfg.K, CALL_INIT) };
        e = f();
    }
#undef CALL_INIT
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(const_partials_kernel, dim3((unsigned)ceil_div(c.ntiles, 256)), dim3(256),
                       0, c.stream, c.partials(), c.ntiles, c.n);
    return hipGetLastError();
}

hipError_t launch_gmm_reweight(Ctx &c, double dalpha, bool reset_check)
{
    const int D = 3 * c.cfg.K - 1;
    const double *llrow = (const double *)c.state_ptr() + (int64_t)D * c.n;
    hipLaunchKernelGGL(gmm_reweight_kernel, dim3((unsigned)c.ntiles), dim3(TPB), 0, c.stream,
                       c.buf.log_weight, llrow, c.buf.scalars, (int)reset_check, dalpha, c.n,
                       c.partials());
    return hipGetLastError();
}

hipError_t launch_gmm_move(Ctx &c, int32_t step, const smc_move_args &a, bool gather_check)
{
    const int W = gmm_waves(c.n, c.cfg.n_data);
    const int sweeps = a.sweeps > 0 ? a.sweeps : (c.cfg.sweeps > 0 ? c.cfg.sweeps : 1);
    bool gather = gather_check;
    for (int s = 0; s < sweeps; ++s) {
        for (int b = 0; b < 3; ++b) {
            if (b == 2 && c.cfg.K == 1)
                continue;
#define CALL_BLOCK(k) dispatch_block<k>(c, W, step, b, s, a.alpha, a.scale[b], gather)
            hipError_t e;
            {
                auto f = [&]() -> hipError_t { SMC_K_SWITCH(c.cfg.K, CALL_BLOCK) };
                e = f();
            }
#undef CALL_BLOCK
            if (e != hipSuccess)
                return e;
            if (gather) {
                c.cur ^= 1;
                gather = false;
            }
        }
    }
    return hipSuccess;
}

hipError_t launch_gmm_loglik_grad(const double *mu, const double *eta, const double *z,
                                  int64_t n, int32_t K, const double *y, int64_t n_data,
                                  double *loglik, double *grad, hipStream_t stream)
{
#define CALL_LL(k) dispatch_loglik<k>(mu, eta, z, n, y, n_data, loglik, grad, stream)
    SMC_K_SWITCH(K, CALL_LL)
#undef CALL_LL
}

}  // namespace smc
