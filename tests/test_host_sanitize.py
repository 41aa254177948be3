"""The library built with AddressSanitizer and UndefinedBehaviorSanitizer on
its host code only (device code is compiled as usual) and driven through its
host-only entry points: the expression parser and generator with valid,
malformed and pseudo-random expressions, size queries and argument
validation (tests/jit_sanitize_check.cpp).  Needs hipcc, no GPU."""

import concurrent.futures
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1105_2279_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["fields.hip", "ape.hip", "batched.hip", "api.cpp", "jit.cpp", "tunecache.cpp"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", *SAN]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_code_is_clean_under_sanitizers(tmp_path):
    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC, *FLAGS, "-x", "hip", "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(HERE, "jit_sanitize_check.cpp")]
    with concurrent.futures.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "jit_sanitize_check")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN[:4], *objs, "-o", exe, "-L/opt/rocm/lib", "-lhiprtc"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr[-3000:]
    assert run.stdout.startswith("ok") and "runtime error" not in run.stderr, run.stdout + run.stderr[-3000:]
