"""Host-side pieces of bench.py: the one-GPU guard, and the rule that HBM
traffic comes from a committed counter summary only while the kernel sources
still hash to the value the summary records; the summaries' commands run
committed files only."""

import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("md,sources", [(bench.APE_COUNTERS_MD, bench.APE_SOURCES),
                                        (bench.HOP_COUNTERS_MD, bench.HOP_SOURCES)], ids=["ape", "hop"])
def test_traffic_only_while_sources_match(md, sources, tmp_path):
    text = open(md).read()
    recorded = re.search(r"source hash: `([0-9a-f]+)`", text).group(1)
    for name in ("f32_12", "f64_18", "f32_18"):
        stored = float(re.search(r"traffic %s: ([0-9.eE+]+)" % name, text).group(1))
        got = bench.measured_traffic(md, sources, name)
        if recorded == bench.kernel_source_hash(sources):
            assert got == stored
        else:
            assert got is None
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(recorded, "0" * len(recorded)))
    assert bench.measured_traffic(str(stale), sources, "f32_12") is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), sources, "f32_12") is None


def test_profile_commands_run_committed_files():
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        text = open(os.path.join(ROOT, "profiles", f)).read()
        cmds = [l for l in text.splitlines() if " rocprofv3 " in l and l.startswith("timeout")]
        assert cmds, f
        for c in cmds:
            assert "-- python3 -u bench.py" in c and "_work" not in c, c


def test_launch_table_covers_benchmark_shapes():
    """The stored launch table holds a geometry for every shape the benchmark
    launches, each one the library's geometry check accepts: the block a
    multiple of 64 (256 or 512 for APE and the batched call, 256 with one
    wave per direction otherwise), an XCD order in 0..2, a t window dividing
    Lt and an LDS tile only for the FP32 APE step."""
    from paper_1105_2279_amd import tuning
    table = tuning.read()
    import latgen

    for op, prec, fmt, L in tuning.SHAPES:
        assert tuning._key(op, prec, fmt, L) in table, (op, prec, fmt, L)
    for prec, fmt in tuning.BATCH_FORMATS:
        assert tuning._key("BATCHED", prec, fmt, latgen.batch_extents()[0]) in table, (prec, fmt)
    for (op, prec, fmt, L), (block, nsite, xcd, tw, lds) in table.items():
        assert (prec, fmt) in (("F32", "LINK12"), ("F64", "LINK18"), ("F32", "LINK18"))
        assert xcd in (0, 1, 2) and tw in (1, 2, 4, 8, 16) and L[3] % tw == 0
        assert lds in ((0, 1, 2, 3, 4) if (op, prec) == ("APE", "F32") else (0,))
        if op == "BATCHED":  # block, groups per ticket
            assert block in (256, 512) and nsite in (1, 2, 4, 8)
        elif op == "APE":
            assert block in (256, 512) and nsite in (1, 2, 4)
        else:
            assert op in ("SHIFT", "CHAIN", "JACOBI") and block == 256 and nsite in (1, 2, 4, 8)


def test_flops_per_link_update_by_hand():
    """Flop per APE link update as the kernels do it, counted by hand: 8 per
    complex FMA, 72 for the combination, 126 for the FP64 projection, 42 per
    row-2 rebuild.  FP32-12 with every product formed per link: 12 products
    of 18 complex FMA and 15 rebuilds (three per lower staple, two per upper
    one); with the backward links staged (LDS tile 2), 13.  With each plane's
    upper product shared (tiles 3 and 4): the lower staples' 6 products, and
    per plane 54 complex FMA (P, then the two upper staples) shared by two
    link updates."""
    assert bench.flops_per_link("f32_12", 0) == 12 * 18 * 8 + 72 + 126 + 15 * 42
    assert bench.flops_per_link("f32_12", 2) == 12 * 18 * 8 + 72 + 126 + 13 * 42
    assert bench.flops_per_link("f32_12", 4) == (6 * 18 + 3 * 54 // 2) * 8 + 72 + 126 + 15 * 42
    assert bench.flops_per_link("f32_12", 3) == (6 * 18 + 3 * 54 // 2) * 8 + 72 + 126 + 13 * 42
    assert bench.flops_per_link("f64_18", 0) == 12 * 18 * 8 + 72 + 126 + 10 * 42
    assert bench.flops_per_link("f32_18", 2) == 12 * 18 * 8 + 72 + 126 + 3 * 42
