"""The resampling entry point that allocates nothing
(smc_resample_weights_noalloc: the library's static per-device scratch as
its workspace) against the entry point with a caller workspace
(smc_resample_weights), through the C ABI: identical summaries and
ancestors on consecutive calls, the second smaller than the first (the
scratch keeps the first call's contents), an error left by one call not
leaking into the next, and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1306_5583_amd import _lib
    _lib.load()
    return _lib


def _lw(n, seed, zeros=0.1):
    rng = np.random.default_rng(seed)
    lw = rng.normal(0.0, 2.5, n) + 40.0
    lw[rng.random(n) < zeros] = -np.inf
    return lw


def _both(L, lw, scheme, threshold=0.5, force=1, seed=99, step=3, problem=1):
    n = lw.size
    s = torch.cuda.current_stream().cuda_stream
    d_lw = torch.as_tensor(lw, device="cuda")
    out = []
    for noalloc in (False, True):
        anc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        sm = torch.full((5,), np.nan, dtype=torch.float64, device="cuda")
        if noalloc:
            L.smc_resample_weights_noalloc(d_lw.data_ptr(), n, scheme, threshold, force, seed,
                                           step, problem, anc.data_ptr(), sm.data_ptr(), s)
        else:
            nb = L.smc_resample_weights_workspace(n, scheme)
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
            L.smc_resample_weights(d_lw.data_ptr(), n, scheme, threshold, force, seed, step,
                                   problem, anc.data_ptr(), sm.data_ptr(), ws.data_ptr(), nb, s)
        torch.cuda.synchronize()
        out.append((anc.cpu().numpy(), sm.cpu().numpy()))
    return out


@pytest.mark.parametrize("scheme,n1", [(1, 1 << 20), (2, 700001), (0, 300000)])
def test_noalloc_matches_workspace_entry_point(L, scheme, n1):
    for call, n in enumerate((n1, 3001)):
        print("noalloc scheme=%d call=%d n=%d" % (scheme, call, n), flush=True)
        (a0, s0), (a1, s1) = _both(L, _lw(n, 7 * n + scheme), scheme, seed=99 + call)
        assert np.array_equal(s0, s1), (call, s0, s1)
        assert s1[3] == 1.0 and s1[4] == 0.0
        assert np.array_equal(a0, a1), call
        assert np.all(np.diff(a1) >= 0) and a1.min() >= 0 and a1.max() < n


def test_error_does_not_leak_into_the_next_call(L):
    # all weights zero: error bits, no ancestors; the next call starts clean
    (a0, s0), (a1, s1) = _both(L, np.full(5000, -np.inf), 1)
    assert np.array_equal(s0[3:], s1[3:]) and s1[3] == 0.0 and s1[4] != 0.0
    assert np.all(a1 == -1)
    (a0, s0), (a1, s1) = _both(L, _lw(4000, 3), 1)
    assert np.array_equal(s0, s1) and s1[4] == 0.0 and np.array_equal(a0, a1)


def test_decision_not_fired_leaves_ancestors(L):
    lw = np.zeros(6000)        # equal weights: ESS = N, never below 0.5 N
    (a0, s0), (a1, s1) = _both(L, lw, 1, force=0)
    assert np.array_equal(s0, s1) and s1[3] == 0.0 and abs(s1[2] - 6000.0) <= 1e-9
    assert np.all(a1 == -1)


def test_size_beyond_the_scratch_is_rejected(L):
    n = 1 << 20   # multinomial needs ~8.1 MiB of workspace, above the 4 MiB array
    assert L.smc_resample_weights_workspace(n, 0) > L.NOALLOC_SCRATCH_BYTES
    lw = torch.zeros(n, dtype=torch.float64, device="cuda")
    anc = torch.zeros(n, dtype=torch.int32, device="cuda")
    sm = torch.zeros(5, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    rc = L.load().smc_resample_weights_noalloc(lw.data_ptr(), n, 0, 0.5, 1, 1, 1, 0,
                                               anc.data_ptr(), sm.data_ptr(), s)
    assert rc == L.SMC_ERR_INVALID_ARG
    with pytest.raises(L.SmcError):
        L.smc_resample_weights_noalloc(lw.data_ptr(), n, 0, 0.5, 1, 1, 1, 0, anc.data_ptr(),
                                       sm.data_ptr(), s)
