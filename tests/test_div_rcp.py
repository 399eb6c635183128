"""The reciprocal-based division of the per-row tap code (div_rcp in the
device header) against the IEEE quotient, for every numerator and
denominator the taps can produce (a C program, about 15 s)."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_div_rcp_equals_ieee_division(tmp_path):
    exe = tmp_path / "div_rcp_check"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", os.path.join(HERE, "div_rcp_check.c"), "-o",
                    str(exe), "-lm"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout
    assert "0 mismatches" in out.stdout
