"""The kernels' site addressing checked on the host (tests/walk_check.cpp):
every site covered once by the 64-site groups, periodic neighbours, and the
t-window, XCD slab-walk and XCD tile orders all bijections, over brick,
linear and ragged lattices.  The check compiles the kernels' own header with
its device functions made host-callable; no GPU."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_site_addressing_and_walks(tmp_path):
    exe = str(tmp_path / "walk_check")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", os.path.join(HERE, "walk_check.cpp"),
                        os.path.join(ROOT, "paper_1105_2279_amd", "csrc", "fields.hip"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.startswith("ok"), run.stdout + run.stderr
