// Host-side accuracy check of the sweep's double-precision elementary
// functions (smc_math.hpp) against long-double references.  Prints the
// maximum error in units of the last place for each function.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

#include "../../paper_1306_5583_amd/csrc/smc_math.hpp"

static double ulp_err(double got, long double ref)
{
    if (std::isinf((double)ref) || std::isinf(got))
        return got == (double)ref ? 0.0 : 1e300;
    const double r = (double)ref;
    const double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    return (double)(std::fabs((long double)got - ref) / (long double)u);
}

int main()
{
    std::mt19937_64 g(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double e_log = 0, e_log_u = 0, e_sin = 0, e_cos = 0, a_sin = 0;
    // log over many binades, and over (0, 1] as in Box-Muller
    for (int i = 0; i < 2000000; ++i) {
        const double x = std::ldexp(0.5 + 0.5 * U(g), (int)(U(g) * 200) - 100);
        e_log = std::fmax(e_log, ulp_err(smc::log_d(x), logl((long double)x)));
        const double u = (double)((g() >> 11) + 1) * 0x1p-53;
        e_log_u = std::fmax(e_log_u, ulp_err(smc::log_d(u), logl((long double)u)));
    }
    // near 1, where cancellation would show
    for (int i = 0; i < 200000; ++i) {
        const double x = 1.0 + (U(g) - 0.5) * 1e-6;
        e_log = std::fmax(e_log, ulp_err(smc::log_d(x), logl((long double)x)));
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < 2000000; ++i) {
        const double x = 2.0 * ((double)((g() >> 11) + 1) * 0x1p-53);   // (0, 2]
        double s, c;
        smc::sincospi_d(x, &s, &c);
        const long double sr = sinl(pi * (long double)x), cr = cosl(pi * (long double)x);
        // absolute error relative to 1 (the values are bounded by 1)
        a_sin = std::fmax(a_sin, (double)std::fmax(std::fabs((long double)s - sr),
                                                    std::fabs((long double)c - cr)));
        if (std::fabs((double)sr) > 1e-3)
            e_sin = std::fmax(e_sin, ulp_err(s, sr));
        if (std::fabs((double)cr) > 1e-3)
            e_cos = std::fmax(e_cos, ulp_err(c, cr));
    }
    double e_exp = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double x = -745.0 * U(g) + (i % 7 == 0 ? 709.0 * U(g) : 0.0);
        const long double ref = expl((long double)x);
        if ((double)ref < 2.3e-308)   // compare normal results in ulp
            continue;
        e_exp = std::fmax(e_exp, ulp_err(smc::exp_d(x), ref));
    }
    for (int i = 0; i < 200000; ++i) {
        const double x = (U(g) - 0.5) * 1e-3;
        e_exp = std::fmax(e_exp, ulp_err(smc::exp_d(x), expl((long double)x)));
    }
    const bool exp_special = smc::exp_d(-INFINITY) == 0.0 && smc::exp_d(0.0) == 1.0 &&
                             std::isinf(smc::exp_d(710.0)) && smc::exp_d(-800.0) == 0.0 &&
                             std::isnan(smc::exp_d(NAN)) &&
                             std::fabs(smc::exp_d(-740.0) - std::exp(-740.0)) <= 1e-320;
    std::printf("exp_ulp %.3f\nexp_special %d\n", e_exp, (int)exp_special);
    double e_exp2 = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double x = i % 5 == 0 ? -U(g) : -1022.0 * U(g);
        e_exp2 = std::fmax(e_exp2, ulp_err(smc::exp2_nonpos(x), exp2l((long double)x)));
    }
    const bool exp2_special = smc::exp2_nonpos(0.0) == 1.0 && smc::exp2_nonpos(-INFINITY) == 0.0 &&
                              smc::exp2_nonpos(-1e300) == 0.0 && smc::exp2_nonpos(-1.0) == 0.5 &&
                              smc::exp2_nonpos(-1074.0) == std::ldexp(1.0, -1074) &&
                              smc::exp2_nonpos(-1080.0) == 0.0;
    std::printf("exp2_ulp %.3f\nexp2_special %d\n", e_exp2, (int)exp2_special);
    const bool special = std::isinf(smc::log_d(0.0)) && smc::log_d(0.0) < 0 &&
                         std::isnan(smc::log_d(-1.0)) && std::isinf(smc::log_d(INFINITY)) &&
                         smc::log_d(1.0) == 0.0 && std::isnan(smc::log_d(NAN));
    std::printf("log_ulp %.3f\nlog_unit_ulp %.3f\nsinpi_ulp %.3f\ncospi_ulp %.3f\nsincospi_abs %.3e\n"
                "special %d\n", e_log, e_log_u, e_sin, e_cos, a_sin, (int)special);
    return 0;
}
