"""Host-side logic of bench.py (no GPU): the single-GPU guard, the roofline
accounting and the matching of committed counter summaries."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_algorithmic_bytes_and_flops_of_the_stratum_kernel():
    import bench
    dims, P, nnz = (4500, 14000, 5), 128, 25_000_000
    # core 10x10x5: records 200 MB, patient rows read and written in every
    # stratum (8 * 4500 * 10 * 128), gene rows once (8 * 14000 * 10)
    r = bench.stratum_roofline("k", "w", False, True, nnz, dims, (10, 10, 5), P, 1e-3)
    assert r["bytes_per_launch"] == pytest.approx(200e6 + 46.08e6 + 1.12e6)
    assert r["achieved"] == pytest.approx(r["bytes_per_launch"] / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    # 6 J1 J2 + 4 (J1 + J2) flops per nonzero
    assert r["alu_tflops"] == pytest.approx(680 * nnz / 1e-3 / 1e12)
    # the multi-launch driver: one stratum per launch
    r1 = bench.stratum_roofline("k", "w", False, False, nnz, dims, (10, 10, 5), P, 1e-3)
    assert r1["bytes_per_launch"] == pytest.approx(200e6 / P + 8 * 4500 * 10 + 1.12e6)
    # the BF16 kernel's matrix-core figures are priced against the BF16 peak
    assert bench.stratum_kernel((20, 20, 5), True, 0, True) == "strata_persistent<20, true, 8>"
    assert bench.stratum_kernel((10, 10, 5), False, 0, False) == "block_step<10>"
    assert bench.stratum_kernel((15, 12, 2), False, 0, True) == "strata_persistent<16, false, 8>"


def test_counter_summaries_match_kernel_workload_and_source(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x_hbm_counters.md").write_text(
        "text\n    kernel_source_sha256: %s\n"
        "    traffic_entry: kA | wl one | 123\n"
        "    traffic_entry: kB | wl one | 456\n" % sha)
    (prof / "x_mfma_counters.md").write_text(
        "    kernel_source_sha256: %s\n    mfma_entry: kA | wl one | 7e9 | 1.5\n" % sha)
    (prof / "old_hbm_counters.md").write_text(
        "    kernel_source_sha256: %s\n    traffic_entry: kC | wl one | 789\n" % ("0" * 64))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.measured_traffic("kA", "wl one") == 123.0
    assert bench.measured_traffic("kB", "wl one") == 456.0
    assert bench.measured_traffic("kA", "wl two") is None
    assert bench.measured_traffic("kC", "wl one") is None  # taken on other source
    assert bench.measured_mfma("kA", "wl one") == (7e9, 1.5)
    r = bench.stratum_roofline("kA", "wl one", True, True, 25_000_000, (4500, 14000, 5), (20, 20, 5), 128, 1e-2)
    assert r["traffic"] == 123.0
    assert r["mfma"]["peak"] == bench.BF16_MFMA_PEAK_TFLOPS
    assert r["mfma"]["tflops"] == pytest.approx(7e9 / 1e-2 / 1e12)
    # a changed source makes every entry stale
    src.write_text("// kernel source, edited\n")
    assert bench.measured_traffic("kA", "wl one") is None
    assert bench.measured_mfma("kA", "wl one") is None
