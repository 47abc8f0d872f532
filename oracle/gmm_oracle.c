/*
 * gmm_oracle.c -- plain FP64 CPU oracle of the tempered Gaussian-mixture SMC
 * sampler (Section 5.2 of the paper: the model of Section 5.2.1, the
 * geometric annealing of Eq. geometry, Algorithm "gmm", the three-block
 * Metropolis random walk and the direct normalising-constant estimate of
 * Eq. smc-ds).
 *
 * TEST INFRASTRUCTURE ONLY (see smc_oracle.c).
 *
 * Parameters are held per particle in unconstrained coordinates
 *   phi = (mu_1..mu_K, eta_1..eta_K, z_1..z_{K-1}),
 * eta_j = log lambda_j (the random walk on the log scale) and
 * z_j = log(omega_j / omega_K) (the random walk on the logit scale; the
 * paper's printed ratio omits the logarithm).  Population arrays are
 * structure-of-arrays [3K-1][n].
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

typedef struct {
    int64_t n;
    uint64_t seed;
    uint32_t problem;
    int32_t K;
    int32_t scheme;
    int32_t move_kind; /* 0: random walk, 1: MALA */
    int32_t sweeps;
    double threshold;
    double mu_mean, mu_sd, gamma_shape, gamma_rate, dir_rho;
} orc_gmm_cfg;

static const double LOG_2PI = 1.8378770664093454835606594728112;
/* columns of the per-step record of orc_gmm_run */
#define ORC_GMM_HIST_COLS 13

/* log omega_j for j = 0..K-1 from the K-1 logits (reference component K). */
static void log_weights(const double *z, int K, double *logw)
{
    double m = 0.0;
    for (int j = 0; j < K - 1; ++j)
        if (z[j] > m)
            m = z[j];
    orc_ksum acc = {0.0, 0.0};
    for (int j = 0; j < K - 1; ++j)
        orc_ks_add(&acc, exp(z[j] - m));
    orc_ks_add(&acc, exp(0.0 - m));
    double lse = m + log(orc_ks_val(&acc));
    for (int j = 0; j < K - 1; ++j)
        logw[j] = z[j] - lse;
    logw[K - 1] = -lse;
}

/*
 * Log-likelihood of the mixture (Section 5.2.1):
 *   l(phi) = sum_k log sum_j omega_j N(y_k | mu_j, 1/lambda_j)
 *          = sum_k lse_j( log omega_j + eta_j/2 - log(2 pi)/2
 *                         - lambda_j (y_k - mu_j)^2 / 2 ),
 * each inner sum taken around its maximum.  When grad is non-NULL it
 * receives dl/dphi (3K-1 values):
 *   dl/dmu_j  = sum_k r_kj lambda_j (y_k - mu_j)
 *   dl/deta_j = sum_k r_kj (1/2 - lambda_j (y_k - mu_j)^2 / 2)
 *   dl/dz_j   = sum_k (r_kj - omega_j),  j < K
 * with responsibilities r_kj = exp(e_kj - lse_j e_kj).
 */
double orc_gmm_loglik_grad(const double *phi, int32_t K, const double *y, int64_t nd,
                           double *grad)
{
    const double *mu = phi, *eta = phi + K, *z = phi + 2 * K;
    double logw[64], c[64], lam[64], e[64];
    log_weights(z, K, logw);
    for (int j = 0; j < K; ++j) {
        lam[j] = exp(eta[j]);
        c[j] = logw[j] + 0.5 * eta[j] - 0.5 * LOG_2PI;
    }
    orc_ksum ll = {0.0, 0.0};
    orc_ksum g[3 * 64];
    int ng = 3 * K - 1;
    for (int q = 0; q < ng; ++q)
        g[q].s = g[q].c = 0.0;
    for (int64_t k = 0; k < nd; ++k) {
        double m = -INFINITY;
        for (int j = 0; j < K; ++j) {
            double d = y[k] - mu[j];
            e[j] = c[j] - 0.5 * lam[j] * d * d;
            if (e[j] > m)
                m = e[j];
        }
        orc_ksum s = {0.0, 0.0};
        for (int j = 0; j < K; ++j)
            orc_ks_add(&s, exp(e[j] - m));
        double Lk = m + log(orc_ks_val(&s));
        orc_ks_add(&ll, Lk);
        if (grad) {
            for (int j = 0; j < K; ++j) {
                double d = y[k] - mu[j];
                double r = exp(e[j] - Lk);
                orc_ks_add(&g[j], r * lam[j] * d);
                orc_ks_add(&g[K + j], r * (0.5 - 0.5 * lam[j] * d * d));
                if (j < K - 1)
                    orc_ks_add(&g[2 * K + j], r - exp(logw[j]));
            }
        }
    }
    if (grad)
        for (int q = 0; q < ng; ++q)
            grad[q] = orc_ks_val(&g[q]);
    return orc_ks_val(&ll);
}

double orc_gmm_loglik(const double *phi, int32_t K, const double *y, int64_t nd)
{
    return orc_gmm_loglik_grad(phi, K, y, nd, NULL);
}

/*
 * Log prior density of phi up to a constant, Jacobians of both changes of
 * variable included (Section 5.2.1 priors):
 *   sum_j -(mu_j - xi)^2 / (2 sd^2)              mu_j ~ N(xi, sd^2)
 * + sum_j (a eta_j - b exp(eta_j))                lambda_j ~ Gamma(a, rate b),
 *                                                 with |d lambda/d eta| = lambda
 * + rho sum_{j=1..K} log omega_j                  omega ~ Dir(rho), with the
 *                                                 log-ratio Jacobian prod omega_j
 */
double orc_gmm_logprior(const orc_gmm_cfg *c, const double *phi)
{
    int K = c->K;
    const double *mu = phi, *eta = phi + K, *z = phi + 2 * K;
    double logw[64];
    log_weights(z, K, logw);
    orc_ksum acc = {0.0, 0.0};
    for (int j = 0; j < K; ++j) {
        double d = mu[j] - c->mu_mean;
        orc_ks_add(&acc, -d * d / (2.0 * c->mu_sd * c->mu_sd));
    }
    for (int j = 0; j < K; ++j)
        orc_ks_add(&acc, c->gamma_shape * eta[j] - c->gamma_rate * exp(eta[j]));
    if (K > 1)
        for (int j = 0; j < K; ++j)
            orc_ks_add(&acc, c->dir_rho * logw[j]);
    return orc_ks_val(&acc);
}

/* Gradient of orc_gmm_logprior:
 *   -(mu_j - xi)/sd^2 ;  a - b exp(eta_j) ;  rho (1 - K omega_j). */
void orc_gmm_logprior_grad(const orc_gmm_cfg *c, const double *phi, double *g)
{
    int K = c->K;
    const double *mu = phi, *eta = phi + K, *z = phi + 2 * K;
    double logw[64];
    log_weights(z, K, logw);
    for (int j = 0; j < K; ++j)
        g[j] = -(mu[j] - c->mu_mean) / (c->mu_sd * c->mu_sd);
    for (int j = 0; j < K; ++j)
        g[K + j] = c->gamma_shape - c->gamma_rate * exp(eta[j]);
    for (int j = 0; j < K - 1; ++j)
        g[2 * K + j] = c->dir_rho * (1.0 - (double)K * exp(logw[j]));
}

static void get_phi(const double *pop, int64_t n, int D, int64_t i, double *phi)
{
    for (int q = 0; q < D; ++q)
        phi[q] = pop[q * n + i];
}

static void put_phi(double *pop, int64_t n, int D, int64_t i, const double *phi)
{
    for (int q = 0; q < D; ++q)
        pop[q * n + i] = phi[q];
}

/*
 * Initialisation from the prior (Algorithm "gmm", initialisation step):
 *   mu_j = xi + sd * n_j        normals: call j/2, element j%2 (tag INIT)
 *   lambda_j = G_j / b          G_j ~ Gamma(a): calls from 64 + 64 j
 *   omega = H / sum(H)          H_j ~ Gamma(rho): calls from 64 + 64*16 + 64 j
 * stored as eta_j = log lambda_j and z_j = log H_j - log H_K.  Fills phi
 * [3K-1][n], the log-likelihood ll[n] and the log prior lp[n].  Returns the
 * number of failed gamma draws.
 */
static int32_t gmm_init_impl(const orc_gmm_cfg *c, const double *y, int64_t nd, double *pop,
                             double *ll, double *lp, const int64_t *ids, int64_t m_ids)
{
    int K = c->K, D = 3 * K - 1;
    int64_t n = ids ? m_ids : c->n;
    int32_t fails = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i) {
        double phi[3 * 64], H[64];
        const uint32_t pid = (uint32_t)(ids ? ids[i] : i);
        for (int j = 0; j < K; j += 2) {
            double z[2];
            orc_normal2(c->seed, pid, 0, ORC_TAG_INIT, (uint32_t)(j / 2), c->problem, z);
            phi[j] = c->mu_mean + c->mu_sd * z[0];
            if (j + 1 < K)
                phi[j + 1] = c->mu_mean + c->mu_sd * z[1];
        }
        for (int j = 0; j < K; ++j) {
            int f = 0;
            double G = orc_gamma(c->seed, pid, 0, ORC_TAG_INIT, (uint32_t)(64 + 64 * j),
                                 c->problem, c->gamma_shape, &f);
            fails += f;
            phi[K + j] = log(G / c->gamma_rate);
        }
        for (int j = 0; j < K; ++j) {
            int f = 0;
            H[j] = orc_gamma(c->seed, pid, 0, ORC_TAG_INIT,
                             (uint32_t)(64 + 64 * 16 + 64 * j), c->problem, c->dir_rho, &f);
            fails += f;
        }
        for (int j = 0; j < K - 1; ++j)
            phi[2 * K + j] = log(H[j]) - log(H[K - 1]);
        put_phi(pop, n, D, i, phi);
        ll[i] = orc_gmm_loglik(phi, K, y, nd);
        lp[i] = orc_gmm_logprior(c, phi);
    }
    return fails;
}

int32_t orc_gmm_init(const orc_gmm_cfg *c, const double *y, int64_t nd, double *pop,
                     double *ll, double *lp)
{
    return gmm_init_impl(c, y, nd, pop, ll, lp, NULL, 0);
}

/* Prior draws of the particles ids[0..m-1] only (column q = particle ids[q]). */
int32_t orc_gmm_init_ids(const orc_gmm_cfg *c, const double *y, int64_t nd, const int64_t *ids,
                         int64_t m, double *pop, double *ll, double *lp)
{
    return gmm_init_impl(c, y, nd, pop, ll, lp, ids, m);
}

/*
 * Reweighting of Algorithm "gmm": lw_i <- (lw_reset ? 0 : lw_i) + dalpha *
 * l(theta_i^{t-1}) (the MCMC-invariant incremental weight of Eq.
 * inc_weight_mcmc for the geometric path).  dalpha == 0 adds exactly 0.
 */
void orc_gmm_reweight(double *lw, const double *ll, int64_t n, double dalpha, int32_t lw_reset)
{
    for (int64_t i = 0; i < n; ++i) {
        double inc = dalpha == 0.0 ? 0.0 : dalpha * ll[i];
        lw[i] = (lw_reset ? 0.0 : lw[i]) + inc;
    }
}

/* tempered log target lp + alpha * l (alpha == 0: the prior alone) */
static double tempered(double lp, double ll, double alpha)
{
    return alpha == 0.0 ? lp : lp + alpha * ll;
}

/*
 * One Metropolis block update of every particle at tempering alpha (the
 * three-block kernel of Section 5.2.1: block 0 = means, 1 = log-precisions,
 * 2 = weight logits).  Random walk: phi'_b = phi_b + scale * n.  MALA:
 * phi'_b = phi_b + scale^2/2 g(phi) + scale * n with g the block gradient of
 * the tempered log target, and the proposal densities enter the ratio.
 * Accept iff log u <= log r, u in (0,1] (tag MH_ACCEPT, call 4*sweep+block).
 * Normals: tag MH_MU/ETA/Z, call 64*sweep + m/2 for block coordinate m.
 * grad ([3K-1][n], likelihood gradient) is required for MALA and may be NULL
 * for the random walk.  accepted[i] (may be NULL) receives 0/1.  Returns the
 * number of accepted proposals.
 */
static int32_t gmm_block_impl(const orc_gmm_cfg *c, uint32_t t, int32_t block, int32_t sweep,
                              double alpha, double scale, const double *y, int64_t nd,
                              double *pop, double *ll, double *lp, double *grad,
                              int32_t *accepted, double *logr_out, double *logu_out,
                              double *scale_out, const int64_t *ids, int64_t m_ids)
{
    int K = c->K, D = 3 * K - 1;
    /* with ids, the arrays hold m_ids particles and column q is particle
       ids[q] (its random numbers are that particle's) */
    int64_t n = ids ? m_ids : c->n;
    int off = block * K;
    int dim = block == 2 ? K - 1 : K;
    uint32_t tag = (uint32_t)(ORC_TAG_MH_MU + block);
    int mala = c->move_kind == 1;
    int32_t count = 0;
    if (dim == 0) {
        if (accepted)
            for (int64_t i = 0; i < n; ++i)
                accepted[i] = 0;
        return 0;
    }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : count)
    for (int64_t i = 0; i < n; ++i) {
        double phi[3 * 64], prop[3 * 64], gl[3 * 64], gp[3 * 64], glp[3 * 64], gpp[3 * 64];
        double xi[64];
        const uint32_t pid = (uint32_t)(ids ? ids[i] : i);
        get_phi(pop, n, D, i, phi);
        for (int m = 0; m < dim; m += 2) {
            double z[2];
            orc_normal2(c->seed, pid, t, tag, (uint32_t)(64 * sweep + m / 2), c->problem, z);
            xi[m] = z[0];
            if (m + 1 < dim)
                xi[m + 1] = z[1];
        }
        double cur = tempered(lp[i], ll[i], alpha);
        memcpy(prop, phi, sizeof(double) * (size_t)D);
        double h2 = scale * scale;
        double drift[64];
        if (mala) {
            get_phi(grad, n, D, i, gl);
            orc_gmm_logprior_grad(c, phi, glp);
            for (int m = 0; m < dim; ++m) {
                double g = glp[off + m] + (alpha == 0.0 ? 0.0 : alpha * gl[off + m]);
                drift[m] = 0.5 * h2 * g;
                prop[off + m] = phi[off + m] + drift[m] + scale * xi[m];
            }
        } else {
            for (int m = 0; m < dim; ++m)
                prop[off + m] = phi[off + m] + scale * xi[m];
        }
        double llp = orc_gmm_loglik_grad(prop, K, y, nd, mala ? gp : NULL);
        double lpp = orc_gmm_logprior(c, prop);
        double logr = tempered(lpp, llp, alpha) - cur;
        /* size of the terms behind log r (for the decision-margin record) */
        double mag = 1.0 + fabs(lp[i]) + fabs(lpp) +
                     (alpha == 0.0 ? 0.0 : alpha * (fabs(ll[i]) + fabs(llp)));
        if (mala) {
            orc_gmm_logprior_grad(c, prop, gpp);
            double fwd = 0.0, bwd = 0.0;
            for (int m = 0; m < dim; ++m) {
                double g2 = gpp[off + m] + (alpha == 0.0 ? 0.0 : alpha * gp[off + m]);
                double a = prop[off + m] - phi[off + m] - drift[m];
                double b = phi[off + m] - prop[off + m] - 0.5 * h2 * g2;
                fwd += a * a;
                bwd += b * b;
            }
            /* log q(phi | phi') - log q(phi' | phi) */
            logr += (fwd - bwd) / (2.0 * h2);
            mag += (fwd + bwd) / (2.0 * h2);
        }
        uint32_t w[4];
        orc_draw_words(c->seed, pid, t, ORC_TAG_MH_ACCEPT, (uint32_t)(4 * sweep + block),
                       c->problem, w);
        double logu = log(orc_u53(w[0], w[1]));
        int acc = logu <= logr;
        if (logr_out)
            logr_out[i] = logr;
        if (logu_out)
            logu_out[i] = logu;
        if (scale_out)
            scale_out[i] = mag;
        if (acc) {
            put_phi(pop, n, D, i, prop);
            ll[i] = llp;
            lp[i] = lpp;
            if (mala)
                put_phi(grad, n, D, i, gp);
            ++count;
        }
        if (accepted)
            accepted[i] = acc;
    }
    return count;
}

int32_t orc_gmm_block(const orc_gmm_cfg *c, uint32_t t, int32_t block, int32_t sweep,
                      double alpha, double scale, const double *y, int64_t nd, double *pop,
                      double *ll, double *lp, double *grad, int32_t *accepted)
{
    return gmm_block_impl(c, t, block, sweep, alpha, scale, y, nd, pop, ll, lp, grad, accepted,
                          NULL, NULL, NULL, NULL, 0);
}

/* Same, also returning log r and log u of every particle's decision. */
int32_t orc_gmm_block_trace(const orc_gmm_cfg *c, uint32_t t, int32_t block, int32_t sweep,
                            double alpha, double scale, const double *y, int64_t nd, double *pop,
                            double *ll, double *lp, double *grad, int32_t *accepted,
                            double *logr_out, double *logu_out)
{
    return gmm_block_impl(c, t, block, sweep, alpha, scale, y, nd, pop, ll, lp, grad, accepted,
                          logr_out, logu_out, NULL, NULL, 0);
}

/* Same for the particles ids[0..m-1] only: the arrays hold m columns,
   column q being particle ids[q] with that particle's random numbers (the
   blocks act on each particle independently, so this equals the columns of
   the whole-population update). */
int32_t orc_gmm_block_trace_ids(const orc_gmm_cfg *c, uint32_t t, int32_t block, int32_t sweep,
                                double alpha, double scale, const double *y, int64_t nd,
                                const int64_t *ids, int64_t m, double *pop, double *ll,
                                double *lp, double *grad, int32_t *accepted, double *logr_out,
                                double *logu_out)
{
    return gmm_block_impl(c, t, block, sweep, alpha, scale, y, nd, pop, ll, lp, grad, accepted,
                          logr_out, logu_out, NULL, ids, m);
}

/* Path-sampling estimate of log(Z_1 / Z_0) (Section 5.2, Eq. path_est): the
   trapezoidal rule over the annealing schedule alpha[0..T] applied to the
   importance-sampling integrands U[0..T] (Eq. path_import), summed in t
   order. */
double orc_path_sampling(const double *alpha, const double *U, int64_t len)
{
    double ps = 0.0;
    for (int64_t t = 1; t < len; ++t)
        ps += 0.5 * (alpha[t] - alpha[t - 1]) * (U[t] + U[t - 1]);
    return ps;
}

/*
 * Complete sampler (Algorithm "gmm") over T tempering steps with
 * alpha[0..T] (alpha[0] = 0) and per-step block scales scales[t][3]
 * (random-walk standard deviations, or MALA step sizes).
 *   step t: dalpha = alpha_t - alpha_{t-1} (0 when alpha_t == 0); reweight;
 *   normalise (dlogZ = L_t - L_{t-1}, L after a resample = log N); resample
 *   when ESS < threshold N; `sweeps` passes of the mu, eta, z blocks at
 *   alpha_t; record.
 * hist[t][0..9] (t = 0..T) = ESS, resampled, dlogZ, logZ, L, accepts of the
 * three blocks, U_t = sum_i W_i l_i (path-sampling integrand, Eq.
 * path_import) and the running path-sampling estimate (Eq. path_est).
 * hist[t][10..12] record how close the step's decisions came to their
 * thresholds, so that a comparison of two independent runs can tell a
 * legitimate rounding-order flip from a mistake:
 *   10: min over the Metropolis decisions of |log r - log u| divided by the
 *       size of the terms behind log r (1 + |lp| + |lp'| + alpha (|l| + |l'|)
 *       + the MALA proposal terms);
 *   11: |ESS - tau N| / (tau N) of the resampling decision (+inf when
 *       tau >= 1 or tau <= 0 decides it);
 *   12: min over the slots of the distance from u_i S to the nearer of the
 *       two cumulative weights bracketing it, divided by S (+inf when the
 *       step does not resample).
 * Final population written to pop_final / lw_final when non-NULL.  Returns
 * the direct estimate log Z (Eq. smc-ds).
 */
double orc_gmm_run(const orc_gmm_cfg *c, const double *y, int64_t nd, int32_t T,
                   const double *alpha, const double *scales, double *hist, double *pop_final,
                   double *lw_final)
{
    int K = c->K, D = 3 * K - 1;
    int64_t n = c->n;
    double *pop = (double *)malloc(sizeof(double) * (size_t)D * (size_t)n);
    double *pop2 = (double *)malloc(sizeof(double) * (size_t)D * (size_t)n);
    double *grad = (double *)calloc((size_t)D * (size_t)n, sizeof(double));
    double *grad2 = (double *)calloc((size_t)D * (size_t)n, sizeof(double));
    double *ll = (double *)malloc(sizeof(double) * (size_t)n);
    double *lp = (double *)malloc(sizeof(double) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
    double *lw = (double *)calloc((size_t)n, sizeof(double));
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *logr = (double *)malloc(sizeof(double) * (size_t)n);
    double *logu = (double *)malloc(sizeof(double) * (size_t)n);
    double *mag = (double *)malloc(sizeof(double) * (size_t)n);
    double *S = (double *)malloc(sizeof(double) * (size_t)n);
    double *us = (double *)malloc(sizeof(double) * (size_t)n);
    orc_gmm_init(c, y, nd, pop, ll, lp);
    if (c->move_kind == 1)
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double phi[3 * 64], g[3 * 64];
            get_phi(pop, n, D, i, phi);
            orc_gmm_loglik_grad(phi, K, y, nd, g);
            put_phi(grad, n, D, i, g);
        }
    double logZ = 0.0, Lprev = log((double)n), a_prev = 0.0;
    int resampled = 0;
    /* path sampling (Section 5.2, Eq. path_est): U_0 is the plain average of
       the log-likelihood over the prior draws (equal weights) */
    orc_ksum u0 = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        orc_ks_add(&u0, ll[i]);
    double U_prev = orc_ks_val(&u0) / (double)n, ps = 0.0, a_alpha_prev_ps = 0.0;
    if (hist) {
        for (int q = 0; q < ORC_GMM_HIST_COLS; ++q)
            hist[q] = 0.0;
        hist[0] = (double)n;
        hist[4] = Lprev;
        hist[8] = U_prev;
        hist[10] = hist[11] = hist[12] = INFINITY;
    }
    for (int32_t t = 1; t <= T; ++t) {
        double a = alpha[t];
        a = a < 1.0 ? a : 1.0;
        a = a > 0.0 ? a : 0.0;
        double dalpha = a == 0.0 ? 0.0 : a - a_prev;
        a_prev = a;
        orc_gmm_reweight(lw, ll, n, dalpha, resampled);
        double nz[3];
        orc_normalise(lw, n, nz);
        double prev = resampled ? log((double)n) : Lprev;
        double dlogz = nz[0] - prev;
        logZ += dlogz;
        Lprev = nz[0];
        resampled = orc_resample_flag(nz[2], n, c->threshold);
        double flag_margin = INFINITY, anc_margin = INFINITY, mh_margin = INFINITY;
        if (c->threshold > 0.0 && c->threshold < 1.0)
            flag_margin = fabs(nz[2] - c->threshold * (double)n) / (c->threshold * (double)n);
        if (resampled) {
            if (orc_resample(c->scheme, c->seed, (uint32_t)t, c->problem, lw, n, anc, S, us) != 0) {
                logZ = NAN;
                break;
            }
            const double tot = S[n - 1];
            for (int64_t i = 0; i < n; ++i) {
                const double x = us[i] * tot;
                const double lo = anc[i] > 0 ? S[anc[i] - 1] : 0.0;
                const double d = fmin(fabs(x - lo), fabs(S[anc[i]] - x)) / tot;
                anc_margin = fmin(anc_margin, d);
            }
            for (int q = 0; q < D; ++q)
                for (int64_t i = 0; i < n; ++i) {
                    pop2[q * n + i] = pop[q * n + anc[i]];
                    grad2[q * n + i] = grad[q * n + anc[i]];
                }
            double *s = pop; pop = pop2; pop2 = s;
            s = grad; grad = grad2; grad2 = s;
            for (int64_t i = 0; i < n; ++i)
                tmp[i] = ll[anc[i]];
            memcpy(ll, tmp, sizeof(double) * (size_t)n);
            for (int64_t i = 0; i < n; ++i)
                tmp[i] = lp[anc[i]];
            memcpy(lp, tmp, sizeof(double) * (size_t)n);
            for (int64_t i = 0; i < n; ++i)
                lw[i] = 0.0;
        }
        int32_t acc[3] = {0, 0, 0};
        for (int s = 0; s < (c->sweeps > 0 ? c->sweeps : 1); ++s)
            for (int b = 0; b < 3; ++b)
            {
                acc[b] += gmm_block_impl(c, (uint32_t)t, b, s, a, scales[3 * t + b], y, nd, pop,
                                         ll, lp, grad, NULL, logr, logu, mag, NULL, 0);
                if (b < 2 || K > 1)
                    for (int64_t i = 0; i < n; ++i)
                        mh_margin = fmin(mh_margin, fabs(logr[i] - logu[i]) / mag[i]);
            }
        /* U_t = sum_i W_t^(i) l(theta_t^(i)) (Eq. path_import: under the
           geometric path the integrand d log q_alpha / d alpha is the
           log-likelihood) and one trapezoid of Eq. path_est */
        double L = resampled ? log((double)n) : nz[0];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            tmp[i] = exp(lw[i] - L) * ll[i];
        orc_ksum u = {0.0, 0.0};
        for (int64_t i = 0; i < n; ++i)
            orc_ks_add(&u, tmp[i]);
        const double U = orc_ks_val(&u);
        ps += 0.5 * (a - a_alpha_prev_ps) * (U + U_prev);
        U_prev = U;
        a_alpha_prev_ps = a;
        if (hist) {
            double *h = hist + ORC_GMM_HIST_COLS * (int64_t)t;
            h[0] = nz[2];
            h[1] = resampled;
            h[2] = dlogz;
            h[3] = logZ;
            h[4] = nz[0];
            h[5] = acc[0];
            h[6] = acc[1];
            h[7] = acc[2];
            h[8] = U;
            h[9] = ps;
            h[10] = mh_margin;
            h[11] = flag_margin;
            h[12] = anc_margin;
        }
    }
    if (pop_final)
        memcpy(pop_final, pop, sizeof(double) * (size_t)D * (size_t)n);
    if (lw_final)
        memcpy(lw_final, lw, sizeof(double) * (size_t)n);
    free(pop); free(pop2); free(grad); free(grad2); free(ll); free(lp); free(tmp); free(lw);
    free(anc); free(logr); free(logu); free(mag); free(S); free(us);
    return logZ;
}
