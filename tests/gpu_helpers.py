"""Shared helpers of the GPU parity tests: tolerance checks that follow the
parity protocol (element-wise relative to the L1 mass of the summands,
ancestors exact except at cumulative-weight boundaries within 1e-12 of the
uniform, decisions exact except within 1e-12 of their threshold)."""
from __future__ import annotations

import math

import numpy as np


def assert_close_l1(got, ref, scale, rtol=1e-12, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), ref.shape)
    same_inf = (got == ref)
    err = np.where(same_inf, 0.0, np.abs(got - ref))
    tol = rtol * np.maximum(1.0, scale)
    bad = ~(err <= tol)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[0]
        raise AssertionError("%s: %d of %d elements outside tolerance; first at %d: got %r ref %r "
                             "tol %r" % (what, int(bad.sum()), bad.size, i, got.ravel()[i],
                                         ref.ravel()[i], tol.ravel()[i]))


def assert_ancestors(anc_gpu, anc_orc, S_orc, u_orc, eps=1e-12, what="ancestors"):
    """Bit-exact except where some cumulative-weight boundary between the two
    answers lies within eps of the uniform (checked on the oracle's S)."""
    anc_gpu = np.asarray(anc_gpu)
    anc_orc = np.asarray(anc_orc)
    assert np.all(np.diff(anc_gpu) >= 0), "%s not sorted" % what
    diff = np.flatnonzero(anc_gpu != anc_orc)
    if diff.size == 0:
        return 0
    tot = S_orc[-1]
    for i in diff:
        lo, hi = sorted((int(anc_gpu[i]), int(anc_orc[i])))
        bounds = S_orc[lo:hi] / tot
        if not np.any(np.abs(bounds - u_orc[i]) <= eps):
            raise AssertionError("%s differ at slot %d: gpu %d oracle %d, nearest boundary %.3e "
                                 "from u" % (what, i, anc_gpu[i], anc_orc[i],
                                             np.min(np.abs(bounds - u_orc[i])) if bounds.size else -1))
    return int(diff.size)


def decision_matches(flag_gpu, flag_orc, value, threshold, eps=1e-12):
    return bool(flag_gpu) == bool(flag_orc) or abs(value - threshold) <= eps * max(1.0, abs(threshold))


# Windows of the parity protocol: a Metropolis decision may differ within
# 1e-11 of the size of log r's terms (the lock-step tests use the same), a
# resampling decision within 1e-12 of tau N, an ancestor within 1e-12 of a
# cumulative-weight boundary.
MH_WINDOW = 1e-11
FLAG_WINDOW = 1e-12
ANC_WINDOW = 1e-12


def first_uncertain_step(hist_o):
    """First step t >= 1 whose decisions (recorded by the oracle's whole run,
    columns 10-12) fall inside a boundary window; len(hist_o) when none do.
    Before it the two runs take identical decisions, so they must agree to
    the protocol's real-valued tolerances."""
    near = ((hist_o[1:, 10] <= MH_WINDOW) | (hist_o[1:, 11] <= FLAG_WINDOW)
            | (hist_o[1:, 12] <= ANC_WINDOW))
    idx = np.flatnonzero(near)
    return int(idx[0]) + 1 if idx.size else hist_o.shape[0]


def assert_gmm_run_matches(h, hist_o, alphas, L, what="run", path=True):
    """Whole mixture-sampler run on the GPU (history h) against the oracle's
    whole run (hist_o from oracle.gmm_run): up to the first step with a
    decision in a boundary window, resampling decisions and accept counts
    exactly, ESS, L, dlogZ, log Z, U_t and the path-sampling estimate within
    1e-12 of the L1 mass of their summands (U_t and the path-sampling
    estimate only with `path`).  Returns that step (T + 1 when every step was
    compared)."""
    ts = first_uncertain_step(hist_o)
    r = slice(1, ts)
    assert np.array_equal(h[r, L.SMC_H_FLAG], hist_o[r, 1]), what + " flags"
    assert np.array_equal(h[r, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3], hist_o[r, 5:8]), \
        "%s accept counts: %s vs %s" % (what, h[r, L.SMC_H_ACC0:L.SMC_H_ACC0 + 3], hist_o[r, 5:8])
    assert_close_l1(h[r, L.SMC_H_ESS], hist_o[r, 0], hist_o[r, 0], 1e-12, what + " ESS")
    assert_close_l1(h[r, L.SMC_H_L], hist_o[r, 4], np.abs(hist_o[r, 4]), 1e-12, what + " L")
    # dlogZ_t = L_t - L_{t-1} (log N after a resample): both terms count
    Lprev = np.where(hist_o[0:ts - 1, 1] != 0, math.log(hist_o[0, 0]), hist_o[0:ts - 1, 4])
    dz_mass = np.abs(hist_o[r, 4]) + np.abs(Lprev)
    assert_close_l1(h[r, L.SMC_H_DLOGZ], hist_o[r, 2], dz_mass, 1e-12, what + " dlogZ")
    assert_close_l1(h[r, L.SMC_H_LOGZ], hist_o[r, 3], np.cumsum(dz_mass), 1e-12, what + " logZ")
    if not path:
        return ts
    U_o = hist_o[:ts, 8]
    assert_close_l1(h[:ts, L.SMC_H_PATH], U_o, np.abs(U_o), 1e-12, what + " U_t")
    a = np.asarray(alphas, dtype=np.float64)[:ts]
    ps_mass = np.concatenate([[0.0], np.cumsum(0.5 * np.diff(a) * (np.abs(U_o[1:]) +
                                                                      np.abs(U_o[:-1])))])
    assert_close_l1(h[:ts, L.SMC_H_PS], hist_o[:ts, 9], ps_mass + np.abs(hist_o[:ts, 9]),
                    1e-12, what + " path sampling")
    return ts
