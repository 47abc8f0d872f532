"""Host-side checks of bench.py's contract (no GPU): more than one GPU is
refused with a message, the committed counter summaries parse, and the
algorithmic byte count per particle."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_profile_values_parse():
    # (a summary whose source digest no longer matches is ignored by bench.py,
    # which then reports the traffic / flops as null)
    v = bench.read_profile_values("pf_move_c1_traffic.txt")
    assert v is not None and float(v["traffic_bytes_per_launch"]) > 0
    assert len(v["source_digest"]) == len(bench.source_digest(bench.PF_MOVE_SOURCES))
    for tag in ("c2", "c3"):
        g = bench.read_profile_values("gmm_block_%s_fp64.txt" % tag)
        assert g is not None and float(g["fp64_flops_per_term"]) > 0


def test_algorithmic_bytes_per_particle():
    # 4 state rows in and out plus the log-weight in and out; right after a
    # resample the old log-weights count as zero and are not read, the
    # 4-byte ancestor index is read instead
    assert bench._bytes_per_particle(False, False) == 80
    assert bench._bytes_per_particle(False, True) == 76
    assert bench._bytes_per_particle(True, False) == 48
    assert bench._bytes_per_particle(True, True) == 44


def test_step_bytes():
    # a whole step: the move, the resampling when it fires (log-weight in,
    # ancestor out: 12 B per particle) and per-tile partials
    n = 1 << 22
    tiles = n // 1024
    assert bench._step_bytes(n, False, True, True) == n * (76 + 12) + tiles * bench.TILE_BYTES
    assert bench._step_bytes(n, False, False, False) == n * 80 + tiles * bench.TILE_BYTES
    assert bench._step_bytes(1000, True, False, True) == 1000 * (48 + 12) + bench.TILE_BYTES
