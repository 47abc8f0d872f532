// smc_math.hpp -- double-precision elementary functions for the per-particle
// sweeps, written for throughput on the vector ALU (no table lookups, no
// branches on the fast path).  Both are textbook constructions:
//
//  log_d(x):   x = 2^e m with m in [sqrt(1/2), sqrt(2)); with s = (m-1)/(m+1)
//              log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...)  (Abramowitz &
//              Stegun 4.1.27), |s| <= 0.1716 so 11 terms reach 1e-18;
//              log x = e ln2 + log m with ln2 split in a high and a low part.
//  exp_d(x):   x = k ln2 + r with k = rint(x / ln2) and |r| <= ln2/2 (Cody &
//              Waite reduction with ln2 in two parts), e^r by its Taylor series
//              to degree 13 (truncation below 5e-18), then scaled by 2^k.
//  exp2_nonpos(x): 2^x for x <= 0 (the terms of a log-sum-exp taken in base
//              2): x = k + r with k = rint(x), |r| <= 1/2 exact, 2^r by the
//              degree-10 minimax polynomial on [-1/2, 1/2] (Remez exchange,
//              2.8e-16 relative error; coefficients from gen_exp2_poly.py),
//              scaled by 2^k.
//  sincospi_d: sin(pi x), cos(pi x) by exact reduction to r = x - n/2,
//              |r| <= 1/4, and the Taylor series of sin(pi r), cos(pi r)
//              to r^17 / r^16 (truncation below 1e-17 for |pi r| <= pi/4),
//              then the
//              quadrant n mod 4.
//
// Accuracy (checked on the host against 50-digit references): a few ulp,
// far inside the 1e-12 relative tolerance of the sweep (2^x: under 4 ulp).  Usable on host and
// device.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace smc {

namespace detail {
// 1/(2k+1), k = 1..12
constexpr double kAtanhC[12] = {1.0 / 3,  1.0 / 5,  1.0 / 7,  1.0 / 9,  1.0 / 11, 1.0 / 13,
                                1.0 / 15, 1.0 / 17, 1.0 / 19, 1.0 / 21, 1.0 / 23, 1.0 / 25};
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double fact(int k) { return k <= 1 ? 1.0 : k * fact(k - 1); }
constexpr double ipow(double x, int k) { return k == 0 ? 1.0 : x * ipow(x, k - 1); }
// sin(pi r) = r * sum_k S_k r^(2k),  S_k = (-1)^k pi^(2k+1) / (2k+1)!
constexpr double sin_c(int k) { return (k % 2 ? -1.0 : 1.0) * ipow(kPi, 2 * k + 1) / fact(2 * k + 1); }
// cos(pi r) = sum_k C_k r^(2k),  C_k = (-1)^k pi^(2k) / (2k)!
constexpr double cos_c(int k) { return (k % 2 ? -1.0 : 1.0) * ipow(kPi, 2 * k) / fact(2 * k); }
constexpr double exp_c(int k) { return 1.0 / fact(k); }
constexpr double kExpC[14] = {exp_c(0), exp_c(1), exp_c(2),  exp_c(3),  exp_c(4),
                              exp_c(5), exp_c(6), exp_c(7),  exp_c(8),  exp_c(9),
                              exp_c(10), exp_c(11), exp_c(12), exp_c(13)};
constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr double kLn2 = 0.69314718055994530941723212145818;
// 2^r ~ sum_j kExp2C[j] r^j on [-1/2, 1/2]: degree-10 minimax in relative
// error (Remez exchange, gen_exp2_poly.py), 2.8e-16 after rounding
constexpr double kExp2C[11] = {
    0x1.0000000000000p+0,  0x1.62e42fefa3a17p-1,  0x1.ebfbdff82c3b9p-3,
    0x1.c6b08d703d48ap-5,  0x1.3b2ab6fbde0f7p-7,  0x1.5d87fe9cc5d6fp-10,
    0x1.4309126056718p-13, 0x1.ffcb55e82f22cp-17, 0x1.62c157ee59177p-20,
    0x1.b6740fc28f781p-24, 0x1.e3991e644e6abp-28};
constexpr double kSinC[10] = {sin_c(0), sin_c(1), sin_c(2), sin_c(3), sin_c(4),
                              sin_c(5), sin_c(6), sin_c(7), sin_c(8), sin_c(9)};
constexpr double kCosC[10] = {cos_c(0), cos_c(1), cos_c(2), cos_c(3), cos_c(4),
                              cos_c(5), cos_c(6), cos_c(7), cos_c(8), cos_c(9)};
// a * b + c with c a wave-uniform constant held in a scalar register pair:
// the fused multiply-add takes it as its scalar operand.  (Left to itself
// the compiler moves each polynomial coefficient into vector registers
// before a two-address multiply-add when the kernel is short of scalar
// registers: two extra vector instructions per coefficient.)
__host__ __device__ inline double fma_k(double a, double b, double c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
#else
    return fma(a, b, c);
#endif
}

// 1 / d for d in [1, 4]: the hardware estimate (exact on the host) refined by
// two Newton steps.
__host__ __device__ inline double recip_1_4(double d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double q = __builtin_amdgcn_rcp(d);
#else
    double q = 1.0 / d;
#endif
    q = fma(q, fma(-d, q, 1.0), q);
    q = fma(q, fma(-d, q, 1.0), q);
    return q;
}
}  // namespace detail

// Natural logarithm of a finite x > 0 (no special-case handling).  The
// atanh series needs 10 terms: the first omitted one is below 1e-18
// relative for |s| <= 0.1716.
constexpr int LOG_TERMS = 10;
__host__ __device__ inline double log_pos_d(double x)
{
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
    const bool lo = m < 0.70710678118654752440;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;  // exact
    // s = f / (2 + f) from a refined reciprocal and one residual correction
    const double d = 2.0 + f;
    const double q = detail::recip_1_4(d);
    double s = f * q;
    s = fma(fma(-s, d, f), q, s);
    const double s2 = s * s;
    double p = detail::kAtanhC[LOG_TERMS - 1];
#pragma unroll
    for (int k = LOG_TERMS - 2; k >= 0; --k)
        p = detail::fma_k(p, s2, detail::kAtanhC[k]);
    // log m = 2s + 2s s^2 p, arranged around f for accuracy: 2s = f - s f
    const double hs = s * f;           // = f - 2s up to rounding
    const double lm = f - (hs - 2.0 * s * s2 * p);
    const double de = (double)e;
    return fma(de, detail::kLn2Hi, fma(de, detail::kLn2Lo, lm));
}

// Natural logarithm; exact special cases: log(0) = -inf, log(inf) = inf,
// log(x < 0) = NaN, NaN propagates.
__host__ __device__ inline double log_d(double x)
{
    double r = log_pos_d(x);
    r = (x == 0.0) ? -INFINITY : r;
    r = (x < 0.0 || x != x) ? __builtin_nan("") : r;
    r = (x == INFINITY) ? INFINITY : r;
    return r;
}

// Exponential of x <= 0 (weights relative to a maximum): x below -1100
// and -inf give 0 through gradual underflow; NaN is not handled.
__host__ __device__ inline double exp_nonpos_d(double x)
{
    const double xc = fmax(x, -1100.0);
    const double k = rint(xc * detail::kLog2e);
    double r = fma(-k, detail::kLn2Hi, xc);
    r = fma(-k, detail::kLn2Lo, r);
    double p = detail::kExpC[13];
#pragma unroll
    for (int j = 12; j >= 0; --j)
        p = detail::fma_k(p, r, detail::kExpC[j]);
    return ldexp(p, (int)k);
}

// Exponential; exp(-inf) = 0, exp(x < -745.2) = 0 (through gradual
// underflow), exp(x > 709.8) = inf, NaN propagates.
__host__ __device__ inline double exp_d(double x)
{
    const double xc = fmin(fmax(x, -1100.0), 1100.0);
    const double k = rint(xc * detail::kLog2e);
    double r = fma(-k, detail::kLn2Hi, xc);
    r = fma(-k, detail::kLn2Lo, r);
    double p = detail::kExpC[13];
#pragma unroll
    for (int j = 12; j >= 0; --j)
        p = fma(p, r, detail::kExpC[j]);
    double v = ldexp(p, (int)k);
    v = (x != x) ? x : v;
    return v;
}

// 2^x for x <= 0: x below -1100 (and -inf) gives 0 through gradual
// underflow; so does NaN (the caller guarantees x is not NaN).  2^0 = 1
// exactly.
__host__ __device__ inline double exp2_nonpos(double x)
{
    const double xc = fmax(x, -1100.0);
    const double k = rint(xc);
    const double r = xc - k;  // exact
    double p = detail::kExp2C[10];
#pragma unroll
    for (int j = 9; j >= 0; --j)
        p = fma(p, r, detail::kExp2C[j]);
    return ldexp(p, (int)k);
}

// 2^x for finite x <= 0 without the lower clamp (device code: the
// exponent conversion saturates): the same value as exp2_nonpos for every
// finite x, one instruction less; -inf or NaN gives NaN, which a caller
// detects and redoes with exp2_nonpos.
__device__ inline double exp2_nonpos_finite(double x)
{
    const double k = rint(x);
    const double r = x - k;  // exact
    double p = detail::kExp2C[10];
#pragma unroll
    for (int j = 9; j >= 0; --j)
        p = fma(p, r, detail::kExp2C[j]);
    return ldexp(p, (int)k);
}

// Square root of a >= 0 that is 0 or at least 2^-767 (device code): the
// hardware reciprocal square-root estimate refined by one Goldschmidt step
// and one residual correction, the same operations and rounding as the
// library square root on that range, without its rescaling of tiny
// arguments and special-case select (0 is the only special value here).
__device__ inline double sqrt_nonneg_d(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = y * 0.5;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, a);
    g = fma(d, h, g);
    const double d2 = fma(-g, g, a);
    g = fma(d2, h, g);
    return a == 0.0 ? a : g;  // sqrt(-0) = -0
}

// sin(pi x) and cos(pi x) for |x| < 2^50 (SMALL: |x| < 2^29, where the
// quadrant index converts to a 32-bit integer in one instruction; the same
// values).
template <bool SMALL = false>
__host__ __device__ inline void sincospi_d(double x, double *sp, double *cp)
{
    const double n = rint(x + x);          // nearest multiple of 1/2
    const double r = fma(n, -0.5, x);      // exact, |r| <= 1/4
    const double r2 = r * r;
    // nine terms each: the first omitted ones are below 1e-17 relative
    double s = detail::kSinC[8];
    double c = detail::kCosC[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        s = detail::fma_k(s, r2, detail::kSinC[k]);
        c = detail::fma_k(c, r2, detail::kCosC[k]);
    }
    s *= r;
    const int q = (SMALL ? (int)n : (int)(long long)n) & 3;
    const double ss = (q & 1) ? c : s;
    const double cc = (q & 1) ? s : c;
    *sp = (q & 2) ? -ss : ss;
    *cp = ((q + 1) & 2) ? -cc : cc;
}

}  // namespace smc
