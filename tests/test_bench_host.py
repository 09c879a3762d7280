"""Host logic of bench.py that needs no GPU: the one-GPU guard, the algorithmic byte counts the
roofline is priced with, the roofline arithmetic over the live kernel timing, and the rule that a
committed counter record counts as `traffic` only while the kernel sources are unchanged."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_algorithmic_bytes_of_the_batched_products():
    n, p, S = 20000, 10000, 256
    # X^T pass: X once in BF16, the BF16 node operands (S x n), the FP32 outputs (S x p)
    assert bench.algorithmic_bytes(2, n, p, 2, S) == 2 * n * p + S * (2 * n + 4 * p)
    assert bench.algorithmic_bytes(2, n, p, 2, S) == pytest.approx(420.48e6)
    # X pass: the operand is S x p in BF16 and the output S x n in FP32
    assert bench.algorithmic_bytes(3, n, p, 2, S) == 2 * n * p + S * (2 * p + 4 * n)
    assert bench.algorithmic_bytes(3, n, p, 2, S) == pytest.approx(425.6e6, rel=1e-3)
    # plain FP64 passes: X once plus the FP64 vectors
    assert bench.algorithmic_bytes(0, n, p, 8, 1) == 8 * n * p + 8 * (3 * n + p)
    assert bench.algorithmic_bytes(1, n, p, 8, 1) == 8 * n * p + 8 * (p + 2 * n)


class _Stats:
    def __init__(self, ms, cnt):
        self.ms, self.cnt = ms, cnt

    def kernel_stats(self, which):
        return self.ms, self.cnt


def test_roofline_from_live_timing():
    n, p, S = 20000, 10000, 256
    # 100 launches of 120 us each
    out = bench.roofline(_Stats(12.0, 100), n, p, 2, S, 2)
    nbytes = bench.algorithmic_bytes(2, n, p, 2, S)
    assert out["bound"] == "hbm" and out["unit"] == "GB/s"
    assert out["peak"] == 8000.0
    assert out["avg_launch_us"] == pytest.approx(120.0)
    assert out["achieved"] == pytest.approx(nbytes / 120e-6 / 1e9, abs=0.05)
    assert out["frac"] == pytest.approx(out["achieved"] / out["peak"], abs=1e-4)
    assert out["launches"] == 100 and out["bytes_per_launch"] == nbytes
    assert out["mfma_context"]["achieved_tflops"] == pytest.approx(2 * n * p * S / 120e-6 / 1e12,
                                                                   abs=0.05)
    assert bench.roofline(_Stats(0.0, 0), n, p, 2, S, 2) is None


def test_traffic_counts_only_for_unchanged_sources(tmp_path, monkeypatch):
    rec = bench.measured_traffic("traffic_bytes_xt_pass")
    if rec is None:
        pytest.skip("the committed counter record does not match the current kernel sources")
    # the committed record: read back unchanged, and plausible against the algorithmic bytes
    alg = bench.algorithmic_bytes(2, 20000, 10000, 2, 256)
    assert alg <= rec <= 1.5 * alg
    # a kernel source that differs from the one the counters were taken on voids the record
    orig = bench.TRAFFIC_SOURCES
    src = tmp_path / "gemm_bf16.h"
    shutil.copy(os.path.join(ROOT, orig[0]), src)
    with open(src, "a") as fh:
        fh.write("\n// changed\n")
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", (str(src),))
    assert bench.measured_traffic("traffic_bytes_xt_pass") is None
    # and so does a missing record
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", orig)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "none.md"))
    assert bench.measured_traffic("traffic_bytes_xt_pass") is None


def test_tiling_codes_and_the_traffic_record():
    # the engine's tiling codes: split-K, plus 100 for the 128-row tile and 200 for the 64-row one
    assert bench.tiling_desc(3) == "256 rows x 256 nodes per workgroup, split-K 3"
    assert bench.tiling_desc(103) == "128 rows x 256 nodes per workgroup, split-K 3"
    assert bench.tiling_desc(201) == "64 rows x 256 nodes per workgroup, split-K 1"
    assert bench.tiling_desc(0) is None  # no engine yet
    rec = bench.measured_traffic("traffic_bytes_xt_pass")
    if rec is None:
        pytest.skip("the committed counter record does not match the current kernel sources")
    # the record holds for the tiling it was taken on, and for no other
    vals = {}
    with open(bench.TRAFFIC_FILE) as fh:
        for line in fh:
            if line.startswith("tiling_xt_pass:"):
                vals["xt"] = int(line.split(":")[1])
    assert bench.measured_traffic("traffic_bytes_xt_pass", tiling=vals["xt"]) == rec
    other = vals["xt"] + 1 if vals["xt"] % 100 < 99 else vals["xt"] - 1
    assert bench.measured_traffic("traffic_bytes_xt_pass", tiling=other) is None
