"""Host-side checks of the benchmark's bookkeeping (no GPU): the algorithmic
byte models behind its roofline fractions, the source-hash gate on the
measured HBM traffic, and the refusal of more than one GPU."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bytes_per_launch_of_the_push_kernels():
    # 64^3 cells, 50 per cell: 96 B per FP64 particle (read + write of six
    # doubles), 56 B mixed (packed cell + six floats, twice), 72 B per cell
    n, c = 13_107_200, 262_144
    assert bench.algorithmic_bytes_per_launch(n, c) == 1_277_165_568
    assert bench.algorithmic_bytes_per_launch(n, c, "mixed") == 752_877_568
    assert bench.algorithmic_bytes_per_launch(0, c) == c * 72


def test_bytes_per_update_of_the_whole_step():
    # state twice, 24 grid passes over 50 particles per cell, re-sort every 20
    assert bench.algorithmic_bytes_per_update(50, 20) == pytest.approx(96 + 3.84 + 6.4)
    assert bench.algorithmic_bytes_per_update(50, 20, "mixed") == pytest.approx(56 + 3.84 + 4.4)
    # more particles per cell and rarer re-sorts approach the particle stream alone
    assert bench.algorithmic_bytes_per_update(1e9, 10**9) == pytest.approx(96, abs=1e-6)
    r = bench.step_roofline(1e9, 50, 20)
    assert r["achieved"] == pytest.approx(106.24)
    assert r["frac"] == pytest.approx(106.24 / 8000.0)
    assert r["unit"] == "GB/s" and r["bound"] == "hbm"


def test_measured_traffic_needs_the_current_kernel_source(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summ = tmp_path / "c.md"
    summ.write_text(f"# title: x\n\n| a | b |\n\nhbm_bytes_per_launch: 1234567\n"
                    f"kernel_source_sha256: {sha}\n")
    assert bench.measured_traffic(str(summ), str(src)) == 1234567.0
    src.write_text("kernel v2\n")                      # source changed since the counters
    assert bench.measured_traffic(str(summ), str(src)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), str(src)) is None


def test_committed_summaries_match_the_committed_sources():
    for counters, src in ((bench.COUNTERS, bench.KERNEL_SRC),
                          (bench.COUNTERS_MIXED, bench.KERNEL_SRC_MIXED),
                          (bench.COUNTERS_SLAB, bench.KERNEL_SRC)):
        t = bench.measured_traffic(counters, src)
        assert t is not None, counters
        assert 1.0e8 < t < 1.0e10


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
