"""The multiply-high division of the kernels' site decoding (FastDiv),
compiled for the host and checked against the hardware integer division
over every divisor up to 4096, large divisors and the top of the numerator
range (tests/fastdiv_check.cpp)."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_fastdiv_matches_division(tmp_path):
    exe = tmp_path / "fastdiv_check"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", os.path.join(HERE, "fastdiv_check.cpp"),
                    "-o", str(exe)], check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert " 0 wrong" in r.stdout
