"""A C program on the C ABI alone (tests/c_abi_check.c): a context created
from a launch-table file launches the stored geometry, saves and re-reads
tables, and refuses malformed ones.  The program is compiled here with the
host C compiler against include/qdpx.h and libqdpx.so."""

import os
import subprocess

import pytest

from gpuhelp import need_gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_1105_2279_amd")


def build_c_check(out):
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(HERE, "c_abi_check.c"), "-o", out, f"-L{PKG}", "-lqdpx", "-L/opt/rocm/lib", "-lamdhip64",
           "-lm", f"-Wl,-rpath,{PKG}", "-Wl,-rpath,/opt/rocm/lib"]
    return subprocess.run(cmd, capture_output=True, text=True)


def test_c_program_compiles_against_the_header(tmp_path):
    r = build_c_check(str(tmp_path / "c_abi_check"))
    assert r.returncode == 0, r.stderr[-3000:]


@pytest.mark.gpu
def test_c_program_launches_stored_geometry(tmp_path):
    need_gpu()
    exe = str(tmp_path / "c_abi_check")
    r = build_c_check(exe)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    env.pop("QDPX_TUNE_CACHE", None)
    run = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=120, env=env)
    assert run.returncode == 0 and run.stdout.strip().endswith("ok"), run.stdout + run.stderr
