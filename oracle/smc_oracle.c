/*
 * smc_oracle.c -- plain FP64 CPU oracle of the SMC sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU library.
 *
 * Every function follows the paper's definitions step by step, in the
 * paper's order, with plain loops, sequential fixed-order (Neumaier
 * compensated) sums and strict IEEE arithmetic (built with -O2
 * -ffp-contract=off, no fast-math).  Loops whose iterations are independent
 * (one particle each: draws, moves, gathers, the terms of a sum) may run on
 * several threads (OpenMP); every sum is still taken by one thread in index
 * order, so the results do not depend on the number of threads.  Citations name the section, equation or
 * algorithm of Zhou, "vSMC: Parallel Sequential Monte Carlo in C++"
 * (arXiv:1306.5583).  Readings of points the paper leaves open are listed in
 * the design notes; each is restated where it is used.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), written here from that definition.
 * Counter = (particle, step, tag<<16 | call, problem); key = (lo32(seed),
 * hi32(seed)).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

/* Threads for the independent loops (the benchmark's CPU baseline times
   one and all); the results are the same for any count. */
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {           /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One Philox call for (particle i, step t, tag, call j, problem p). */
static void draw(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                 uint32_t p, uint32_t w[4])
{
    uint32_t ctr[4] = {i, t, (tag << 16) | (j & 0xFFFFu), p};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, w);
}

void orc_draw_words(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                    uint32_t p, uint32_t *w)
{
    draw(seed, i, t, tag, j, p, w);
}

/* Uniform on (0,1] from the top 53 bits of the 64-bit word (a:b). */
double orc_u53(uint32_t a, uint32_t b)
{
    uint64_t bits = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(bits + 1u) * 0x1p-53;
}

/* Uniform on (0,1] in single precision from one word. */
float orc_u24(uint32_t w)
{
    return (float)((w >> 8) + 1u) * 0x1p-24f;
}

static const double TWO_PI = 6.283185307179586476925286766559;

/* Two standard normals from one call (Box-Muller). */
static void normal2(const uint32_t w[4], double z[2])
{
    double u1 = orc_u53(w[0], w[1]);
    double u2 = orc_u53(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    double th = TWO_PI * u2;
    z[0] = r * cos(th);
    z[1] = r * sin(th);
}

/* Four single-precision standard normals from one call (Box-Muller). */
static void normal4f(const uint32_t w[4], float z[4])
{
    const float two_pi_f = 6.28318530717958647692f;
    for (int h = 0; h < 2; ++h) {
        float u1 = orc_u24(w[2 * h]);
        float u2 = orc_u24(w[2 * h + 1]);
        float r = sqrtf(-2.0f * logf(u1));
        float th = two_pi_f * u2;
        z[2 * h] = r * cosf(th);
        z[2 * h + 1] = r * sinf(th);
    }
}

void orc_normal2(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                 uint32_t p, double *z)
{
    uint32_t w[4];
    draw(seed, i, t, tag, j, p, w);
    normal2(w, z);
}

void orc_normal4f(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t j,
                  uint32_t p, float *z)
{
    uint32_t w[4];
    draw(seed, i, t, tag, j, p, w);
    normal4f(w, z);
}

/*
 * Gamma(shape, 1) variate from calls jbase, jbase+1, ...
 *   shape == 1 : -log u, u from call jbase (exponential).
 *   shape  > 1 : Marsaglia & Tsang (2000); attempt k uses call jbase+1+2k for
 *                the normal and call jbase+2+2k for the uniform.
 *   shape  < 1 : Gamma(shape+1) from the same attempts, times u^(1/shape)
 *                with u from call jbase.
 * At most 31 attempts; *fail is set when all are rejected (returns NaN).
 */
double orc_gamma(uint64_t seed, uint32_t i, uint32_t t, uint32_t tag, uint32_t jbase,
                 uint32_t p, double shape, int *fail)
{
    uint32_t w[4];
    if (shape == 1.0) {
        draw(seed, i, t, tag, jbase, p, w);
        return -log(orc_u53(w[0], w[1]));
    }
    double a = shape < 1.0 ? shape + 1.0 : shape;
    double d = a - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    double g = NAN;
    for (int k = 0; k < 31; ++k) {
        double z[2];
        draw(seed, i, t, tag, jbase + 1 + 2 * k, p, w);
        normal2(w, z);
        double v = 1.0 + c * z[0];
        if (v <= 0.0)
            continue;
        v = v * v * v;
        draw(seed, i, t, tag, jbase + 2 + 2 * k, p, w);
        double u = orc_u53(w[0], w[1]);
        if (log(u) < 0.5 * z[0] * z[0] + d - d * v + d * log(v)) {
            g = d * v;
            break;
        }
    }
    if (isnan(g)) {
        if (fail)
            *fail = 1;
        return g;
    }
    if (shape < 1.0) {
        draw(seed, i, t, tag, jbase, p, w);
        g *= pow(orc_u53(w[0], w[1]), 1.0 / shape);
    }
    return g;
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation in index order                          */
/* ------------------------------------------------------------------------ */
typedef orc_ksum ksum;
#define ks_add orc_ks_add
#define ks_val orc_ks_val

/* ------------------------------------------------------------------------ */
/* Weights: log-sum-exp, ESS, normalising-constant increment (Section 2.1,  */
/* the ESS definition; Section 2.2, the ratio Z_t / Z_{t-1}).               */
/* ------------------------------------------------------------------------ */

double orc_max(const double *x, int64_t n)
{
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (x[i] > m)
            m = x[i];
    return m;
}

/* log sum_i exp(scale * lw_i), computed around the maximum. */
static double lse_scaled(const double *lw, int64_t n, double scale)
{
    double m = orc_max(lw, n);
    if (m == -INFINITY)
        return -INFINITY;
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        e[i] = exp(scale * (lw[i] - m));
    ksum acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        ks_add(&acc, e[i]);
    free(e);
    return scale * m + log(ks_val(&acc));
}

double orc_lse(const double *lw, int64_t n) { return lse_scaled(lw, n, 1.0); }

/*
 * Normalisation summary of unnormalised log-weights lw:
 *   out[0] = L  = log sum_i exp(lw_i)
 *   out[1] = L2 = log sum_i exp(2 lw_i)
 *   out[2] = ESS = 1 / sum_i W_i^2 = exp(2L - L2), W_i = exp(lw_i - L)
 */
void orc_normalise(const double *lw, int64_t n, double *out)
{
    double L = lse_scaled(lw, n, 1.0);
    double L2 = lse_scaled(lw, n, 2.0);
    out[0] = L;
    out[1] = L2;
    out[2] = exp(2.0 * L - L2);
}

/*
 * Resampling decision (Section 4.1, sampler construction): resample when
 * ESS/N is below the threshold; threshold >= 1 always, <= 0 never.
 */
int orc_resample_flag(double ess, int64_t n, double threshold)
{
    if (threshold >= 1.0)
        return 1;
    if (threshold <= 0.0)
        return 0;
    return ess < threshold * (double)n;
}

/* ------------------------------------------------------------------------ */
/* Resampling (Section 2.1, replication counts R_i with sum N; Eq. resample) */
/* ------------------------------------------------------------------------ */
enum { ORC_RS_MULTINOMIAL = 0, ORC_RS_SYSTEMATIC = 1, ORC_RS_STRATIFIED = 2 };

/*
 * Ordered uniforms u_0 <= ... <= u_{N-1} in (0,1]:
 *   systematic : u_i = (i + U) / N, U from call (0, t, RESAMPLE<<16, p)
 *   stratified : u_i = (i + U_i) / N, U_i from call (i, t, RESAMPLE<<16, p)
 *   multinomial: u_i = G_i / G_N with G_i = E_0 + ... + E_i, E_k = -log v_k,
 *                v_k from call (k, t, RESAMPLE<<16 | 1, p), k = 0..N; these
 *                are the order statistics of N iid uniforms.
 */
void orc_resample_uniforms(int scheme, uint64_t seed, uint32_t t, uint32_t p, int64_t n,
                           double *u)
{
    uint32_t w[4];
    if (scheme == ORC_RS_SYSTEMATIC) {
        draw(seed, 0, t, ORC_TAG_RESAMPLE, 0, p, w);
        double U = orc_u53(w[0], w[1]);
        for (int64_t i = 0; i < n; ++i)
            u[i] = ((double)i + U) / (double)n;
    } else if (scheme == ORC_RS_STRATIFIED) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t wi[4];
            draw(seed, (uint32_t)i, t, ORC_TAG_RESAMPLE, 0, p, wi);
            u[i] = ((double)i + orc_u53(wi[0], wi[1])) / (double)n;
        }
    } else {
        double *G = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        double *E = (double *)malloc(sizeof(double) * (size_t)(n + 1));
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k <= n; ++k) {
            uint32_t wk[4];
            draw(seed, (uint32_t)k, t, ORC_TAG_RESAMPLE, 1, p, wk);
            E[k] = -log(orc_u53(wk[0], wk[1]));
        }
        ksum acc = {0.0, 0.0};
        for (int64_t k = 0; k <= n; ++k) {
            ks_add(&acc, E[k]);
            G[k] = ks_val(&acc);
        }
        free(E);
        for (int64_t i = 0; i < n; ++i)
            u[i] = G[i] / G[n];
        free(G);
    }
}

/*
 * Ancestors from ordered uniforms.  S_j = sum_{k<=j} exp(lw_k - m) (m = max
 * lw, compensated running sum), S = S_{N-1}.  a_i = min{ j : S_j > u_i * S };
 * when no such j exists, a_i is the last j with S_j > S_{j-1} (S_{-1} = 0),
 * so a zero-weight particle is never chosen.  The output is non-decreasing.
 * S (length N) is written to S_out when non-NULL.  Returns 0, or -1 when all
 * weights are zero or not finite.
 */
int orc_ancestors(const double *lw, int64_t n, const double *u, int32_t *anc,
                  double *S_out)
{
    double m = orc_max(lw, n);
    if (!(m > -INFINITY) || !isfinite(m))
        return -1;
    double *S = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        S[j] = exp(lw[j] - m);
    ksum acc = {0.0, 0.0};
    for (int64_t j = 0; j < n; ++j) {
        ks_add(&acc, S[j]);
        S[j] = ks_val(&acc);
    }
    double tot = S[n - 1];
    if (!(tot > 0.0) || !isfinite(tot)) {
        free(S);
        return -1;
    }
    int64_t last = 0;
    for (int64_t j = 0; j < n; ++j)
        if (S[j] > (j ? S[j - 1] : 0.0))
            last = j;
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) {
        double x = u[i] * tot;
        /* u is non-decreasing, so the search resumes where it stopped */
        while (j < n && !(S[j] > x))
            ++j;
        anc[i] = (int32_t)(j < n ? j : last);
        if (j >= n)
            j = n; /* stays exhausted for the remaining slots */
    }
    if (S_out)
        memcpy(S_out, S, sizeof(double) * (size_t)n);
    free(S);
    return 0;
}

/* Full resampling step (every scheme): its ordered uniforms, then the
 * inverse of the cumulative weights at each of them. */
int orc_resample(int scheme, uint64_t seed, uint32_t t, uint32_t p, const double *lw,
                 int64_t n, int32_t *anc, double *S_out, double *u_out)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    orc_resample_uniforms(scheme, seed, t, p, n, u);
    int rc = orc_ancestors(lw, n, u, anc, S_out);
    if (u_out)
        memcpy(u_out, u, sizeof(double) * (size_t)n);
    free(u);
    return rc;
}

/*
 * In-place parent layout of Section 4.1 (value collection copy): copy_from[i]
 * is the parent of slot i and a particle that survives keeps its own slot
 * (copy_from[j] == j).  Derived from the sorted ancestors: survivors keep
 * their slot; extra copies fill the empty slots in ascending order.
 */
void orc_copy_from(const int32_t *anc, int64_t n, int32_t *copy_from)
{
    int32_t *R = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i)
        R[anc[i]]++;
    for (int64_t i = 0; i < n; ++i)
        copy_from[i] = R[i] > 0 ? (int32_t)i : -1;
    int64_t slot = 0;
    for (int64_t j = 0; j < n; ++j) {
        for (int32_t c = 1; c < R[j]; ++c) {
            while (copy_from[slot] >= 0)
                ++slot;
            copy_from[slot] = (int32_t)j;
        }
    }
    free(R);
}

/* ------------------------------------------------------------------------ */
/* Importance-sampling estimate (Section 2.1, phi_hat_3; Section 4.1,        */
/* monitors): est_c = sum_i W_i h_c(x_i), W_i = exp(lw_i - L).               */
/* x is structure-of-arrays [dim][n].                                         */
/* ------------------------------------------------------------------------ */
void orc_weighted_mean(const double *x, int64_t dim, const double *lw, int64_t n,
                       double *est)
{
    double L = orc_lse(lw, n);
    double *W = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        W[i] = exp(lw[i] - L);
    for (int64_t c = 0; c < dim; ++c) {
        ksum acc = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i)
            ks_add(&acc, W[i] * x[c * n + i]);
        est[c] = ks_val(&acc);
    }
    free(W);
}

/* ------------------------------------------------------------------------ */
/* Tracking particle filter (Section 5.1, Algorithm "pf")                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    uint64_t seed;
    uint32_t problem;
    int32_t fp32_state;       /* 1: single-precision state and draws */
    int32_t paper_compatible; /* 1: drop the Student-t normalising constant */
    int32_t scheme;
    double threshold;
    double dt, sd_pos, sd_vel, obs_scale, obs_nu; /* obs_nu = inf: Gaussian */
    double init_sd[4];
} orc_pf_cfg;

/*
 * Observation log-density of one coordinate given the position.  Student-t
 * with nu degrees of freedom and scale s:
 *   C - (nu+1)/2 * log1p(((y - pos)/s)^2 / nu),
 *   C = lgamma((nu+1)/2) - lgamma(nu/2) - log(nu*pi)/2 - log s
 * (C dropped when paper_compatible, as in the paper's listing).  Gaussian
 * (nu infinite): -log(2 pi s^2)/2 - (y - pos)^2 / (2 s^2).
 */
double orc_pf_obs_logdens(const orc_pf_cfg *c, double pos, double y)
{
    double s = c->obs_scale;
    double r = (y - pos) / s;
    if (isinf(c->obs_nu))
        return -0.5 * log(TWO_PI * s * s) - 0.5 * r * r;
    double nu = c->obs_nu;
    double C = 0.0;
    if (!c->paper_compatible)
        C = lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(nu * M_PI) - log(s);
    return C - 0.5 * (nu + 1.0) * log1p(r * r / nu);
}

static double pf_loglik(const orc_pf_cfg *c, double px, double py, const double y[2])
{
    return orc_pf_obs_logdens(c, px, y[0]) + orc_pf_obs_logdens(c, py, y[1]);
}

/*
 * Initialisation: x_0 ~ N(0, diag(init_sd^2)); lw_0 = log L(x_0 | y_0).
 * FP64 draws: call 0 -> (x_pos, y_pos), call 1 -> (x_vel, y_vel).
 * FP32 draws: call 0 -> all four.  x is [4][n] in double even for the FP32
 * variant (it then holds float-representable values).
 */
void orc_pf_init(const orc_pf_cfg *c, const double y0[2], double *x, double *lw)
{
    int64_t n = c->n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xi[4];
        if (c->fp32_state) {
            float z[4];
            orc_normal4f(c->seed, (uint32_t)i, 0, ORC_TAG_INIT, 0, c->problem, z);
            for (int k = 0; k < 4; ++k)
                xi[k] = (double)((float)c->init_sd[k] * z[k]);
        } else {
            double z[4];
            orc_normal2(c->seed, (uint32_t)i, 0, ORC_TAG_INIT, 0, c->problem, z);
            orc_normal2(c->seed, (uint32_t)i, 0, ORC_TAG_INIT, 1, c->problem, z + 2);
            for (int k = 0; k < 4; ++k)
                xi[k] = c->init_sd[k] * z[k];
        }
        for (int k = 0; k < 4; ++k)
            x[k * n + i] = xi[k];
        lw[i] = pf_loglik(c, xi[0], xi[1], y0);
    }
}

/*
 * One move of Algorithm "pf" at step t on an already-resampled population:
 *   pos <- pos + dt * vel + sd_pos * n ;  vel <- vel + sd_vel * n
 * (positions use the old velocity), then
 *   lw_out = (lw_reset ? 0 : lw_in) + log L(x_t | y_t).
 * FP64 draws: call 0 -> position noise, call 1 -> velocity noise (tag
 * PF_MOVE, step t).  FP32: one call, four float normals.
 */
void orc_pf_move(const orc_pf_cfg *c, uint32_t t, const double yt[2], const double *x_in,
                 const double *lw_in, int lw_reset, double *x_out, double *lw_out)
{
    int64_t n = c->n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double px = x_in[0 * n + i], py = x_in[1 * n + i];
        double vx = x_in[2 * n + i], vy = x_in[3 * n + i];
        if (c->fp32_state) {
            float z[4];
            orc_normal4f(c->seed, (uint32_t)i, t, ORC_TAG_PF_MOVE, 0, c->problem, z);
            float dt = (float)c->dt, sp = (float)c->sd_pos, sv = (float)c->sd_vel;
            float fpx = (float)px, fpy = (float)py, fvx = (float)vx, fvy = (float)vy;
            float npx = (fpx + dt * fvx) + sp * z[0];
            float npy = (fpy + dt * fvy) + sp * z[1];
            float nvx = fvx + sv * z[2];
            float nvy = fvy + sv * z[3];
            px = npx; py = npy; vx = nvx; vy = nvy;
        } else {
            double z[4];
            orc_normal2(c->seed, (uint32_t)i, t, ORC_TAG_PF_MOVE, 0, c->problem, z);
            orc_normal2(c->seed, (uint32_t)i, t, ORC_TAG_PF_MOVE, 1, c->problem, z + 2);
            double npx = (px + c->dt * vx) + c->sd_pos * z[0];
            double npy = (py + c->dt * vy) + c->sd_pos * z[1];
            double nvx = vx + c->sd_vel * z[2];
            double nvy = vy + c->sd_vel * z[3];
            px = npx; py = npy; vx = nvx; vy = nvy;
        }
        x_out[0 * n + i] = px;
        x_out[1 * n + i] = py;
        x_out[2 * n + i] = vx;
        x_out[3 * n + i] = vy;
        double inc = pf_loglik(c, px, py, yt);
        lw_out[i] = (lw_reset ? 0.0 : lw_in[i]) + inc;
    }
}

/* x_out[k][i] = x_in[k][anc[i]] (value-collection copy, Section 4.1). */
void orc_gather(const double *x_in, int64_t dim, int64_t n, const int32_t *anc,
                double *x_out)
{
    for (int64_t k = 0; k < dim; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            x_out[k * n + i] = x_in[k * n + anc[i]];
    }
}

/*
 * Complete filter over T observations y[T][2] (Algorithm "pf"): initialise at
 * t = 0, then T-1 moves.  After the weighting of every step (t = 0
 * included): normalise, resample when the rule says so, then record the
 * importance-sampling estimate of all four state components.
 *   hist[t][0..8] = ESS, resampled flag, dlogZ, logZ, L, mean x_pos, y_pos,
 *                   x_vel, y_vel.
 * log Z_0 = L_0 - log N; dlogZ_t = L_t - L_{t-1}, with L_{t-1} = log N after
 * a resample (Section 2.2, the ratio estimator with normalised previous
 * weights).  Returns log Z (NaN on a numeric failure).
 */
double orc_pf_run(const orc_pf_cfg *c, int32_t T, const double *y, double *hist,
                  double *x_final, double *lw_final)
{
    int64_t n = c->n;
    double *x = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    double *x2 = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    double *lw = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double logZ = 0.0, Lprev = 0.0;
    int resampled = 0;
    for (int32_t t = 0; t < T; ++t) {
        if (t == 0) {
            orc_pf_init(c, y, x, lw);
        } else {
            orc_pf_move(c, (uint32_t)t, y + 2 * t, x, lw, resampled, x2, lw);
            double *tmp = x; x = x2; x2 = tmp;
        }
        double nz[3];
        orc_normalise(lw, n, nz);
        double prev = (t == 0 || resampled) ? log((double)n) : Lprev;
        double dlogz = nz[0] - prev;
        logZ += dlogz;
        Lprev = nz[0];
        resampled = orc_resample_flag(nz[2], n, c->threshold);
        if (resampled) {
            if (orc_resample(c->scheme, c->seed, (uint32_t)t, c->problem, lw, n, anc, NULL,
                             NULL) != 0) {
                logZ = NAN;
                break;
            }
            orc_gather(x, 4, n, anc, x2);
            double *tmp = x; x = x2; x2 = tmp;
            for (int64_t i = 0; i < n; ++i)
                lw[i] = 0.0;
        }
        double *h = hist ? hist + 9 * (int64_t)t : NULL;
        if (h) {
            h[0] = nz[2];
            h[1] = resampled;
            h[2] = dlogz;
            h[3] = logZ;
            h[4] = nz[0];
            orc_weighted_mean(x, 4, lw, n, h + 5);
        }
    }
    if (x_final)
        memcpy(x_final, x, sizeof(double) * 4 * (size_t)n);
    if (lw_final)
        memcpy(lw_final, lw, sizeof(double) * (size_t)n);
    free(x); free(x2); free(lw); free(anc);
    return logZ;
}

/* ------------------------------------------------------------------------ */
/* Batch helpers for statistical checks of the transforms: draws for        */
/* particles i = 0..n-1 at one (step, tag, call).                            */
/* ------------------------------------------------------------------------ */
void orc_fill_normals(uint64_t seed, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                      int64_t n, double *out /* 2n */)
{
    for (int64_t i = 0; i < n; ++i)
        orc_normal2(seed, (uint32_t)i, t, tag, j, p, out + 2 * i);
}

void orc_fill_normals_f32(uint64_t seed, uint32_t t, uint32_t tag, uint32_t j, uint32_t p,
                          int64_t n, float *out /* 4n */)
{
    for (int64_t i = 0; i < n; ++i)
        orc_normal4f(seed, (uint32_t)i, t, tag, j, p, out + 4 * i);
}

void orc_fill_gamma(uint64_t seed, uint32_t t, uint32_t tag, uint32_t jbase, uint32_t p,
                    double shape, int64_t n, double *out, int32_t *fails)
{
    int f = 0;
    for (int64_t i = 0; i < n; ++i)
        out[i] = orc_gamma(seed, (uint32_t)i, t, tag, jbase, p, shape, &f);
    *fails = f;
}
