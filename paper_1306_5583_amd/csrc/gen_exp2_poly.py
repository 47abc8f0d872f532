"""Coefficients of the polynomial behind smc::exp2_nonpos (smc_math.hpp).

p(r) is the degree-10 minimax approximation of 2^r on [-1/2, 1/2] in
relative error, found by the Remez exchange algorithm at 60 significant
digits (start: Chebyshev extrema; new reference: the alternating extrema of
the error on a 4000-point grid) and rounded to double.  Prints the C array
and the relative error of the rounded polynomial on a 20000-point grid at
60 digits.  Run: python gen_exp2_poly.py
"""
import mpmath as mp

DEG = 10


def remez(deg=DEG, iters=30, grid_n=4000):
    mp.mp.dps = 60
    f = lambda r: mp.power(2, r)
    a, b = mp.mpf(-0.5), mp.mpf(0.5)
    n = deg + 2
    xs = [(a + b) / 2 - (b - a) / 2 * mp.cos(mp.pi * k / (n - 1)) for k in range(n)]
    grid = [a + (b - a) * k / grid_n for k in range(grid_n + 1)]
    c = None
    for _ in range(iters):
        # p(x_i) - f(x_i) = (-1)^i E f(x_i) at the reference points
        A = mp.matrix(n, n)
        rhs = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = -((-1) ** i) * f(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        c = [sol[j] for j in range(deg + 1)]
        vals = [(sum(c[j] * x ** j for j in range(deg + 1)) - f(x)) / f(x) for x in grid]
        ext = [0] + [k for k in range(1, grid_n)
                     if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0] + [grid_n]
        pts = []
        for k in ext:
            if pts and (vals[k] > 0) == (vals[pts[-1]] > 0):
                if abs(vals[k]) > abs(vals[pts[-1]]):
                    pts[-1] = k
            else:
                pts.append(k)
        while len(pts) > n:
            pts.pop(0 if abs(vals[pts[0]]) < abs(vals[pts[-1]]) else -1)
        if len(pts) < n:
            break
        xs = [grid[k] for k in pts]
    return [float(v) for v in c]


def max_rel_error(cd, points=20000):
    mp.mp.dps = 60
    worst = mp.mpf(0)
    for i in range(points + 1):
        r = mp.mpf(-0.5) + mp.mpf(i) / points
        p = mp.mpf(0)
        for cj in reversed(cd):
            p = p * r + mp.mpf(cj)
        worst = max(worst, abs(p / mp.power(2, r) - 1))
    return float(worst)


if __name__ == "__main__":
    cd = remez()
    print("constexpr double kExp2C[%d] = {" % len(cd))
    for v in cd:
        print("    %s,  // %.17g" % (float.hex(v), v))
    print("};")
    print("// max relative error of the rounded polynomial: %.3g" % max_rel_error(cd))
