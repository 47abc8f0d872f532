"""Accuracy of the sweep's own double-precision log, exp, 2^x and sin/cos(pi x)
(paper_1306_5583_amd/csrc/smc_math.hpp), compiled for the host and checked
against long-double references over millions of arguments."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_math_functions_within_few_ulp(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "math_check")
    subprocess.run([hipcc, "-O2", "-o", exe, os.path.join(HERE, "support", "math_check.cpp")],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(line.split() for line in out.strip().splitlines())
    assert float(vals["log_ulp"]) < 4.0
    assert float(vals["log_unit_ulp"]) < 4.0
    assert float(vals["sinpi_ulp"]) < 4.0
    assert float(vals["cospi_ulp"]) < 4.0
    assert float(vals["sincospi_abs"]) < 5e-16
    assert vals["special"] == "1"
    assert float(vals["exp_ulp"]) < 4.0
    assert vals["exp_special"] == "1"
    assert float(vals["exp2_ulp"]) < 4.0
    assert vals["exp2_special"] == "1"
