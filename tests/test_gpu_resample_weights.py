"""GPU parity of the one-shot resampling entry point (smc_resample_weights:
caller-held log-weights in, normalisation summary and sorted ancestors out)
against the oracle's normalisation and resampling (Section 2.1; Eq.
resample), for every scheme, ragged sizes, zero weights, the decision rule
and the error path."""
import numpy as np
import pytest

from gpu_helpers import assert_ancestors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCHEMES = {"multinomial": 0, "systematic": 1, "stratified": 2}


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1306_5583_amd import _lib
    _lib.load()
    return _lib


def _weights(n, seed, zeros=0.0):
    rng = np.random.default_rng(seed)
    lw = rng.normal(0.0, 3.0, n) - 700.0          # far from 0: the max shift matters
    if zeros:
        lw[rng.random(n) < zeros] = -np.inf
    return lw


def _run(L, lw, scheme, threshold=0.5, force=0, seed=17, step=5, problem=0, anc_init=None):
    n = lw.size
    d_lw = torch.as_tensor(lw, device="cuda")
    anc = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    if anc_init is not None:
        anc.copy_(torch.as_tensor(anc_init, dtype=torch.int32))
    summary = torch.zeros(5, dtype=torch.float64, device="cuda")
    nb = L.smc_resample_weights_workspace(n, SCHEMES[scheme])
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.smc_resample_weights(d_lw.data_ptr(), n, SCHEMES[scheme], threshold, force, seed, step,
                           problem, anc.data_ptr(), summary.data_ptr(), ws.data_ptr(), nb,
                           torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return anc.cpu().numpy().astype(np.int64), summary.cpu().numpy()


@pytest.mark.parametrize("scheme", list(SCHEMES))
@pytest.mark.parametrize("n", [1, 1000, 70001, 1 << 20])
def test_matches_oracle(L, orc, scheme, n):
    lw = _weights(n, n + len(scheme), zeros=0.2 if n > 1 else 0.0)
    anc, sm = _run(L, lw, scheme, force=1, seed=17, step=5, problem=3)
    Lo, L2o, esso = orc.normalise(lw)
    assert abs(sm[0] - Lo) <= 1e-12 * max(1.0, abs(Lo))
    assert abs(sm[1] - L2o) <= 1e-12 * max(1.0, abs(L2o))
    assert abs(sm[2] - esso) <= 1e-12 * esso
    assert sm[3] == 1.0 and sm[4] == 0.0
    anc_o, S_o, u_o = orc.resample(scheme, 17, 5, lw, p=3)
    assert_ancestors(anc, anc_o, S_o, u_o, what="%s n=%d" % (scheme, n))
    assert np.all(np.isfinite(lw[anc]))           # zero weights are never chosen


def test_decision_rule(L, orc):
    n = 5000
    lw = _weights(n, 3)
    _, _, ess = orc.normalise(lw)
    assert ess < 0.5 * n
    # ESS below threshold N: resample; above: ancestors untouched
    anc, sm = _run(L, lw, "systematic", threshold=1.2 * ess / n)
    assert sm[3] == 1.0
    keep = np.arange(n)
    anc, sm = _run(L, lw, "systematic", threshold=0.5 * ess / n, anc_init=keep)
    assert sm[3] == 0.0 and np.array_equal(anc, keep)
    anc, sm = _run(L, lw, "systematic", threshold=0.0, anc_init=keep)   # never
    assert sm[3] == 0.0 and np.array_equal(anc, keep)
    anc, sm = _run(L, lw, "systematic", threshold=1.0)                  # always
    assert sm[3] == 1.0
    anc_o, S_o, u_o = orc.resample("systematic", 17, 5, lw)
    assert_ancestors(anc, anc_o, S_o, u_o)


def test_all_zero_weights_report_an_error(L):
    lw = np.full(3000, -np.inf)
    keep = np.arange(3000)
    anc, sm = _run(L, lw, "systematic", force=1, anc_init=keep)
    assert sm[3] == 0.0 and sm[4] != 0.0
    assert np.array_equal(anc, keep)


def test_invalid_arguments(L):
    from paper_1306_5583_amd import SmcError
    lw = torch.zeros(100, dtype=torch.float64, device="cuda")
    anc = torch.zeros(100, dtype=torch.int32, device="cuda")
    sm = torch.zeros(5, dtype=torch.float64, device="cuda")
    nb = L.smc_resample_weights_workspace(100, 1)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(SmcError):      # workspace too small
        L.smc_resample_weights(lw.data_ptr(), 100, 1, 0.5, 1, 1, 1, 0, anc.data_ptr(),
                               sm.data_ptr(), ws.data_ptr(), nb - 1, s)
    with pytest.raises(SmcError):      # unknown scheme
        L.smc_resample_weights(lw.data_ptr(), 100, 9, 0.5, 1, 1, 1, 0, anc.data_ptr(),
                               sm.data_ptr(), ws.data_ptr(), nb, s)
    with pytest.raises(SmcError):      # misaligned log-weights
        L.smc_resample_weights(lw.data_ptr() + 8, 99, 1, 0.5, 1, 1, 1, 0, anc.data_ptr(),
                               sm.data_ptr(), ws.data_ptr(), nb, s)
