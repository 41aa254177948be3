"""The launch-table file reader and writer checked on the host
(tests/tunecache_check.cpp): round trip, other architectures, missing and
malformed files.  No GPU."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


# host code only: AddressSanitizer and UndefinedBehaviorSanitizer, no recovery
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan_ubsan"])
def test_table_file_reader_and_writer(tmp_path, sanitize):
    exe = str(tmp_path / "tunecache_check")
    r = subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        *(SAN if sanitize else []), os.path.join(HERE, "tunecache_check.cpp"),
                        os.path.join(ROOT, "paper_1105_2279_amd", "csrc", "tunecache.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    run = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0 and run.stdout.startswith("ok"), run.stdout + run.stderr[-3000:]
    assert "runtime error" not in run.stderr, run.stderr[-3000:]
