"""Coefficients of the polynomial behind smc::exp2_nonpos (smc_math.hpp).

p(r) interpolates 2^r at the 12 Chebyshev nodes of [-1/2, 1/2] (degree 11),
solved at 50 significant digits and rounded to double.  Prints the C array
and the interpolation error of the rounded polynomial (relative, measured on
a dense grid at 50 digits).  Run: python gen_exp2_poly.py
"""
import mpmath as mp


def coefficients(deg=11, dps=50):
    mp.mp.dps = dps
    n = deg + 1
    nodes = [mp.mpf(1) / 2 * mp.cos(mp.pi * (2 * k + 1) / (2 * n)) for k in range(n)]
    a = mp.matrix([[x ** j for j in range(n)] for x in nodes])
    b = mp.matrix([mp.power(2, x) for x in nodes])
    c = mp.lu_solve(a, b)
    return [float(c[j]) for j in range(n)]


def max_rel_error(cd, points=4000):
    worst = mp.mpf(0)
    for i in range(points + 1):
        r = mp.mpf(-0.5) + mp.mpf(i) / points
        p = mp.mpf(0)
        for cj in reversed(cd):
            p = p * r + mp.mpf(cj)
        worst = max(worst, abs(p / mp.power(2, r) - 1))
    return float(worst)


if __name__ == "__main__":
    cd = coefficients()
    print("constexpr double kExp2C[%d] = {" % len(cd))
    for j, v in enumerate(cd):
        print("    %s,%s" % (float.hex(v), "  // %.17g" % v))
    print("};")
    print("// max relative interpolation error: %.3g" % max_rel_error(cd))
