"""CPU checks of bench.py's contract: the one-GPU guard, the algorithmic byte
counts the roofline divides by, and the hash gate on the committed HBM
counter summary."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_algorithmic_bytes_per_launch():
    # one window: counts read + written (8 S), neighbours (16), couplings
    # (32) and N_A V (8) per tet, plus 8 per nonzero (tet, species, face) move
    assert bench.window_bytes(996_564, 15, 0.0) == 996_564 * 176
    assert bench.window_bytes(1, 1, 3.0) == 64 + 24
    # detect kernel: counts (4 S), N_A V (8), region label only with regions
    assert bench.detect_kernel_bytes(480_000, 10, 1) == 480_000 * 48
    assert bench.detect_kernel_bytes(10, 15, 2) == 10 * 69


def test_roofline_fields():
    kt = {"windows": 10, "main_ms": 4.0, "detect_ms": 0.2}
    r = bench.roofline(1000, 15, 2, 10, 5000, kt, "test", "dendrite_calcium15")
    b = 1000 * 176 + 8 * 500
    assert r["bytes_per_launch"] == b
    assert r["achieved"] == b / 0.4e-3 / 1e9
    assert r["frac"] == r["achieved"] / 8000.0
    assert r["window"]["main_us"] == 400.0 and r["window"]["detect_us"] == 20.0
    assert set(("bound", "achieved", "peak", "unit", "frac", "traffic")) <= set(r)


def test_record_kernel_bytes():
    # counts (4 S per tet), plus the region label only with regions
    assert bench.record_kernel_bytes(996_564, 15, 2) == 996_564 * 61
    assert bench.record_kernel_bytes(480_000, 10, 1) == 480_000 * 40


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel text")
    sha = hashlib.sha256(b"kernel text").hexdigest()
    summary = tmp_path / "counters.txt"
    summary.write_text("# comment: ignored\n"
                       f"kernel_source_sha256: {sha}\n"
                       "FETCH_SIZE_KiB_per_dispatch: 100\nWRITE_SIZE_KiB_per_dispatch: 50\n"
                       "fetch_factor: 2.0\nwrite_factor: 1.0\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "COUNTERS", {"w": str(summary)})
    assert bench.measured_traffic("w") == pytest.approx((100 * 2.0 + 50) * 1024.0)
    src.write_bytes(b"kernel text, changed")
    assert bench.measured_traffic("w") is None



def test_valu_issue_only_for_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel text")
    sha = hashlib.sha256(b"kernel text").hexdigest()
    summary = tmp_path / "sq.txt"
    summary.write_text("# window_main_kernel<16, 24>  2856  1.0  2.0\n"
                       "window_main_kernel<16, 24>        2856   349872576.4\n"
                       f"kernel_source_sha256: {sha}\n"
                       "window_main_kernel_SQ_INSTS_VALU_per_dispatch: 614400\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "SQ_COUNTERS", {"dendrite_calcium15": str(summary)})
    monkeypatch.setattr(bench, "TRACES", {"dendrite_calcium15": str(tmp_path / "none.txt")})
    monkeypatch.setattr(bench, "COUNTERS", {"dendrite_calcium15": str(tmp_path / "none.txt")})
    assert bench.measured_valu() == 614400.0
    # 1024 SIMDs x 2.4 GHz / 4 cycles: 614.4e9 wave64 instructions per second
    assert bench.VALU_PEAK_PER_S == pytest.approx(614.4e9)
    kt = {"windows": 1, "main_ms": 1e-3, "detect_ms": 1e-3}  # 1 us per launch
    r = bench.roofline(1000, 15, 2, 1, 0, kt, "test", "dendrite_calcium15")
    assert r["valu_issue"]["frac"] == pytest.approx(614400 / 1e-6 / 614.4e9)
    src.write_bytes(b"kernel text, changed")
    assert bench.measured_valu() is None
    assert "valu_issue" not in bench.roofline(1000, 15, 2, 1, 0, kt, "test", "dendrite_calcium15")
