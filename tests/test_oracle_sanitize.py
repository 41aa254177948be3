"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host compiler only) and driven through every entry point on small ragged
lattices with one and four threads (tests/oracle_sanitize_check.c): no
out-of-bounds access, leak or undefined operation is reported."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize_check"
    build = subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                            os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_sanitize_check.c"),
                            "-lm", "-o", str(exe)], capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("sanitizer runtime not available: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.strip() == "ok" and "runtime error" not in r.stderr, r.stdout + r.stderr[-3000:]
