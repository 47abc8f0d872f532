"""Shared helpers of the GPU parity tests: tolerance checks that follow the
parity protocol (element-wise relative to the L1 mass of the summands,
ancestors exact except at cumulative-weight boundaries within 1e-12 of the
uniform, decisions exact except within 1e-12 of their threshold)."""
from __future__ import annotations

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
