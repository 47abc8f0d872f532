"""Pins of the oracle's weight algebra (Section 2.1 ESS, Section 2.2 ratio
estimator) and resampling (Section 2.1 replication counts; Eq. resample)."""
import math

import mpmath
import numpy as np
import pytest


def test_lse_constant_vector(orc):
    for n, c in [(1, 0.0), (7, -3.5), (1000, 12.25)]:
        L, L2, ess = orc.normalise(np.full(n, c))
        assert L == pytest.approx(c + math.log(n), abs=1e-13)
        assert L2 == pytest.approx(2 * c + math.log(n), abs=1e-13)
        assert ess == pytest.approx(n, rel=1e-12)


def test_ess_one_hot(orc):
    lw = np.full(50, -np.inf)
    lw[17] = 3.0
    L, L2, ess = orc.normalise(lw)
    assert L == 3.0 and L2 == 6.0 and ess == 1.0


def test_ess_two_level_by_hand(orc):
    # k particles with weight a, n-k with weight b (unnormalised)
    n, k, a, b = 10, 3, 2.0, 0.5
    lw = np.log(np.array([a] * k + [b] * (n - k)))
    tot = k * a + (n - k) * b
    W = np.array([a] * k + [b] * (n - k)) / tot
    L, L2, ess = orc.normalise(lw)
    assert L == pytest.approx(math.log(tot), abs=1e-14)
    assert ess == pytest.approx(1.0 / float((W ** 2).sum()), rel=1e-14)


def test_dlogz_against_mpmath(orc):
    # log Z_t/Z_{t-1} = log sum_i W_{t-1,i} exp(inc_i) (Section 2.2)
    rng = np.random.default_rng(3)
    n = 600
    lw = rng.normal(0, 3, n)
    inc = rng.normal(-2, 4, n)
    d = orc.lse(lw + inc) - orc.lse(lw)
    mpmath.mp.dps = 50
    lw_m = [mpmath.mpf(float(v)) for v in lw]
    inc_m = [mpmath.mpf(float(v)) for v in inc]
    Z0 = mpmath.fsum(mpmath.exp(v) for v in lw_m)
    ratio = mpmath.fsum(mpmath.exp(a) / Z0 * mpmath.exp(b) for a, b in zip(lw_m, inc_m))
    assert abs(d - float(mpmath.log(ratio))) <= 1e-13 * max(1.0, abs(d))


def test_resample_flag_rule(orc):
    assert orc.resample_flag(10.0, 100, 1.0) is True       # threshold >= 1: always
    assert orc.resample_flag(100.0, 100, 1.5) is True
    assert orc.resample_flag(1.0, 100, 0.0) is False       # threshold <= 0: never
    assert orc.resample_flag(49.999, 100, 0.5) is True     # strictly below
    assert orc.resample_flag(50.0, 100, 0.5) is False


# ------------------------------------------------------------- resampling

SCHEMES = ["systematic", "multinomial", "stratified"]


def _counts(anc, n):
    return np.bincount(anc, minlength=n)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ancestors_sorted_and_sum_to_n(orc, scheme):
    rng = np.random.default_rng(11)
    for n in [1, 2, 3, 64, 1000, 4097]:
        lw = rng.normal(0, 2, n)
        anc, S, u = orc.resample(scheme, 1234, 5, lw)
        assert anc.dtype == np.int32 and anc.size == n
        assert np.all(np.diff(anc) >= 0)
        assert _counts(anc, n).sum() == n
        assert anc.min() >= 0 and anc.max() < n
        assert np.all(np.diff(u) >= 0) and u[0] > 0 and u[-1] <= 1


@pytest.mark.parametrize("scheme", SCHEMES)
def test_zero_weights_never_chosen(orc, scheme):
    rng = np.random.default_rng(12)
    n = 500
    lw = rng.normal(0, 1, n)
    dead = rng.random(n) < 0.6
    lw[dead] = -np.inf
    for t in range(20):
        anc, _, _ = orc.resample(scheme, 99, t, lw)
        assert not np.any(dead[anc])


def test_all_zero_weights_rejected(orc):
    with pytest.raises(FloatingPointError):
        orc.resample("systematic", 1, 0, np.full(10, -np.inf))


def test_systematic_counts_floor_ceil(orc):
    # each R_j is floor(N W_j) or ceil(N W_j) for systematic resampling
    rng = np.random.default_rng(13)
    for trial in range(30):
        n = int(rng.integers(2, 3000))
        lw = rng.normal(0, 1.5, n)
        anc, S, u = orc.resample("systematic", 77, trial, lw)
        R = _counts(anc, n)
        NW = n * np.exp(lw - orc.lse(lw))
        assert np.all(R >= np.floor(NW - 1e-9)) and np.all(R <= np.ceil(NW + 1e-9))


def test_systematic_is_inverse_cdf(orc):
    # a_i is the first index whose cumulative normalised weight exceeds (i+U)/N
    rng = np.random.default_rng(14)
    n = 300
    lw = rng.normal(0, 1, n)
    w = np.exp(lw - lw.max())
    cdf = np.cumsum(w) / w.sum()
    anc, S, u = orc.resample("systematic", 5, 2, lw)
    U = u[0] * n
    assert np.allclose(u, (np.arange(n) + U) / n, rtol=0, atol=1e-15)
    ref = np.searchsorted(cdf, u, side="right")
    ref = np.minimum(ref, n - 1)
    assert np.array_equal(anc, ref)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_counts_unbiased(orc, scheme):
    # E[R_j] = N W_j (Eq. resample with M = N and equal new weights)
    n, reps = 64, 20000
    rng = np.random.default_rng(15)
    lw = rng.normal(0, 1.0, n)
    W = np.exp(lw - orc.lse(lw))
    tot = np.zeros(n)
    tot2 = np.zeros(n)
    for r in range(reps):
        anc, _, _ = orc.resample(scheme, 31337, r, lw)
        R = _counts(anc, n)
        tot += R
        tot2 += R * R
    mean = tot / reps
    var = tot2 / reps - mean ** 2
    se = np.sqrt(np.maximum(var, 1e-12) / reps)
    z = (mean - n * W) / se
    assert np.all(np.abs(z) < 5.5)
    if scheme == "multinomial":
        # Var R_j = N W_j (1 - W_j)
        expected = n * W * (1 - W)
        assert np.all(np.abs(var - expected) < 0.1 * expected + 0.02)


def test_copy_from_layout(orc):
    rng = np.random.default_rng(16)
    n = 200
    lw = rng.normal(0, 2, n)
    anc, _, _ = orc.resample("systematic", 8, 1, lw)
    cf = orc.copy_from(anc)
    R = _counts(anc, n)
    # survivors keep their own slot; the multiset of parents is unchanged
    assert np.all(cf[R > 0] == np.nonzero(R > 0)[0])
    assert np.array_equal(np.sort(cf), anc)
    # the empty slots, in ascending order, take the extra copies in
    # ascending (parent, copy) order: the sorted ancestors minus the first
    # copy of each parent
    extras = anc[1:][anc[1:] == anc[:-1]]
    assert np.array_equal(cf[R == 0], extras)


def test_weighted_mean(orc):
    rng = np.random.default_rng(17)
    x = rng.normal(size=(3, 100))
    lw = rng.normal(size=100)
    W = np.exp(lw) / np.exp(lw).sum()
    est = orc.weighted_mean(x, lw)
    assert np.allclose(est, x @ W, rtol=1e-13, atol=1e-15)


def test_ties_go_right_and_clamp(orc):
    # equal weights: S_j = j + 1 exactly; uniforms on the boundaries
    n = 8
    lw = np.zeros(n)
    u = (np.arange(n) + 1.0) / n
    anc, S = orc.ancestors(lw, u)
    assert np.array_equal(S, np.arange(1.0, n + 1))
    # a_i = min{j : S_j > u_i S}: a tie moves to the next index; u = 1 has no
    # such j and falls back to the last positive-weight particle
    assert list(anc) == list(range(1, n)) + [n - 1]
    lw2 = lw.copy()
    lw2[-3:] = -np.inf          # last positive weight is index n-4
    anc2, S2 = orc.ancestors(lw2, np.full(n, 1.0))
    assert np.all(anc2 == n - 4)


def test_systematic_counts_closed_form_exact(orc):
    # The oracle takes a_i = min{j : S_j > u_i S} at u_i = (i + U)/N.  In
    # exact arithmetic that gives particle j the replication number
    # R_j = c(S_j) - c(S_{j-1}) with c(x) = #{i : (i + U)/N < x/S} =
    # ceil(N x / S - U) clamped to [0, N] (Section 2.1's counts, a different
    # route to the same integers), checked here in rational arithmetic on
    # the oracle's own cumulative weights (slots past the last count go to
    # the last positive weight); only counts whose argument lies within
    # 1e-12 of an integer may round the other way
    from fractions import Fraction
    rng = np.random.default_rng(21)
    for trial in range(12):
        n = int(rng.integers(3, 400))
        lw = rng.normal(0, 2.0, n)
        lw[rng.random(n) < 0.2] = -np.inf
        if not np.isfinite(lw).any():
            lw[0] = 0.0
        anc, S, u = orc.resample("systematic", 99, trial, lw)
        w = orc.draw_words(99, 0, trial, 7, 0)     # the step's systematic U
        U = Fraction(orc.u53(w[0], w[1]))
        tot = Fraction(float(S[-1]))
        R = _counts(anc, n)
        prev = 0
        near = set()
        for j in range(n):
            x = Fraction(float(S[j])) * n / tot - U
            c = min(n, max(0, -((-x.numerator) // x.denominator)))
            if abs(float(x) - round(float(x))) < 1e-12 * n:
                near.add(j)
            exp_r = c - prev
            if j not in near and (j == 0 or j - 1 not in near):
                pos = np.nonzero(np.isfinite(lw))[0]
                if j != pos[-1]:
                    assert R[j] == exp_r, (trial, j, R[j], exp_r)
            prev = c
        assert R.sum() == n
