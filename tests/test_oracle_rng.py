"""Pins of the oracle's random-number layer: Philox4x32-10 words against the
generator's published known-answer vectors and against rocRAND's engine
(run, not copied), and the distribution of the derived uniforms, normals
and gamma variates."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for r in rows:
        out = orc.philox(r[0:4], r[4:6])
        assert [int(v) for v in out] == r[6:10]


@pytest.fixture(scope="module")
def rocrand_words(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rr_words")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "golden", "rocrand_philox_words.cpp")],
                   check=True, capture_output=True)

    def run(queries):
        text = "\n".join(" ".join("%08x" % v for v in q) for q in queries) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [[int(v, 16) for v in line.split()] for line in out.strip().splitlines()]
    return run


def test_philox_matches_rocrand_engine(orc, rocrand_words):
    rng = np.random.default_rng(0)
    queries = []
    for _ in range(400):
        c0 = int(rng.integers(0, 2 ** 32))
        c1 = int(rng.integers(0, 2 ** 20))        # steps stay far below 2^30
        c2 = int(rng.integers(0, 2 ** 32))
        c3 = int(rng.integers(0, 2 ** 32))
        k0 = int(rng.integers(0, 2 ** 32))
        k1 = int(rng.integers(0, 2 ** 32))
        queries.append((c0, c1, c2, c3, k0, k1))
    ref = rocrand_words(queries)
    for q, r in zip(queries, ref):
        assert [int(v) for v in orc.philox(q[:4], q[4:])] == r


def test_counter_layout(orc):
    # counter = (particle, step, tag<<16 | call, problem), key = (lo, hi) of the seed
    seed = 0x1234567890ABCDEF
    w = orc.draw_words(seed, 7, 11, 3, 5, 9)
    ref = orc.philox([7, 11, (3 << 16) | 5, 9], [seed & 0xFFFFFFFF, seed >> 32])
    assert list(w) == list(ref)


def test_u53_exact_range(orc):
    assert orc.u53(0, 0) == 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    # the low 11 bits of the second word are discarded
    assert orc.u53(5, 0x7FF) == orc.u53(5, 0)
    assert orc.u53(0, 0x800) == 2 * 2.0 ** -53
    assert orc.u53(1, 0) == (2.0 ** 21 + 1) * 2.0 ** -53


def test_u24_exact_range(orc):
    assert orc.u24(0) == np.float32(2.0 ** -24)
    assert orc.u24(0xFFFFFFFF) == np.float32(1.0)
    assert orc.u24(0x1FF) == np.float32(2 * 2.0 ** -24)


def test_normals_distribution(orc):
    z = orc.fill_normals(2024, 3, 2, 0, 500_000)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two outputs of one call are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / np.sqrt(z.size / 2)


def test_normals_f32_distribution(orc):
    z = orc.fill_normals_f32(99, 1, 2, 0, 250_000).astype(np.float64)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4


@pytest.mark.parametrize("shape", [1.0, 0.4, 2.0, 5.5])
def test_gamma_distribution(orc, shape):
    g, fails = orc.fill_gamma(17, 0, 1, 64, shape, 200_000)
    assert fails == 0
    assert stats.kstest(g, "gamma", args=(shape,)).pvalue > 1e-4
    assert abs(g.mean() - shape) < 5 * np.sqrt(shape / g.size)


def test_gamma_shape_one_is_exponential_of_first_call(orc):
    g, _ = orc.gamma(5, 3, 0, 1, 64, 1.0)
    w = orc.draw_words(5, 3, 0, 1, 64)
    assert g == -np.log(orc.u53(int(w[0]), int(w[1])))
