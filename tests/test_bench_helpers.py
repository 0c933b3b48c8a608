"""Host logic of bench.py (no GPU): the roofline arithmetic, the counter
summaries keyed by kernel, workload, precision and source hash, the recorded
full-size oracle run, and the single-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_roofline_arithmetic():
    dom = {"count": 4, "ms": 0.4, "bytes": 4 * 800e6, "bytes_csr": 4 * 1000e6}
    r = bench.roofline_of(dom, "k", 840e6, {"timed_one_launch_in": 16})
    # 800 MB per 100 us launch = 8000 GB/s = the peak
    assert r["avg_us"] == pytest.approx(100.0)
    assert r["achieved"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(1.0)
    assert r["csr_model"]["achieved"] == pytest.approx(10000.0)
    assert r["traffic_over_algorithmic"] == pytest.approx(1.05)
    assert r["traffic_frac"] == pytest.approx(1.05)
    assert r["timed_one_launch_in"] == 16
    empty = bench.roofline_of({"count": 0, "ms": 0.0, "bytes": 0.0}, "k", None)
    assert empty["frac"] == 0.0 and empty["traffic"] is None


def _write_summary(path, sha, bytes_per_launch):
    with open(path, "w") as fh:
        fh.write("# summary\n\nsome text: with a colon\n")
        fh.write(f"kernel_source_sha256_16: {sha}\n")
        fh.write(f"hbm_bytes_per_launch: {bytes_per_launch}\n")


def test_traffic_keyed_by_kernel_workload_precision_and_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "traffic_file",
                        lambda k, w, p: str(tmp_path / f"traffic_{k}_{w}_{p}.txt"))
    assert bench.read_traffic("k_cg_spmv", "cube3d_128", "fp64") is None   # not measured
    _write_summary(tmp_path / "traffic_k_cg_spmv_cube3d_128_fp64.txt", bench.kernel_hash(), 398e6)
    assert bench.read_traffic("k_cg_spmv", "cube3d_128", "fp64") == pytest.approx(398e6)
    assert bench.read_traffic("k_cg_spmv", "cube3d_128", "mixed") is None   # other precision
    assert bench.read_traffic("k_cg_spmv", "cube3d_64", "fp64") is None     # other workload
    # taken on other sources: not reported
    _write_summary(tmp_path / "traffic_k_cg_spmv_cube3d_128_fp64.txt", "0" * 16, 398e6)
    assert bench.read_traffic("k_cg_spmv", "cube3d_128", "fp64") is None
    # the batch kernels hash their own sources
    _write_summary(tmp_path / "traffic_kb_rows_batch2d_512_fp64.txt", bench.kernel_hash("batch"), 4e8)
    assert bench.read_traffic("kb_rows", "batch2d_512", "fp64", group="batch") == pytest.approx(4e8)
    assert bench.read_traffic("kb_rows", "batch2d_512", "fp64") is None


def test_kernel_hash_covers_the_sources():
    for group, files in bench.KERNEL_SOURCES.items():
        assert len(bench.kernel_hash(group)) == 16
        for f in files:
            assert os.path.exists(os.path.join(bench.CSRC, f)), f
    assert bench.kernel_hash("single") != bench.kernel_hash("batch")


def test_recorded_full_size_oracle_run():
    rec = bench.recorded_cpu_baseline(128)
    assert rec is not None and rec["recorded"] and rec["kind"] == "oracle"
    assert rec["value"] == pytest.approx(2048383 / rec["seconds"], rel=1e-3)
    assert rec["cores"] >= 1
    assert bench.recorded_cpu_baseline(7) is None


def test_paper_context_is_the_published_a3_times():
    ctx = bench.paper_context()
    s = ctx["seconds"]
    # Tables Tab:S5_cube_times_mustang / _wolf, case A3: TRON1..3 slow down as
    # the inner tolerance tightens, and the faster core is faster everywhere
    for core in ("mustang_1_core", "wolf_1_core"):
        t = s[core]
        assert t["galerkin"] < t["tron1"] < t["tron2"] < t["tron3"] < t["blmvm"]
    for k in s["wolf_1_core"]:
        assert s["wolf_1_core"][k] < s["mustang_1_core"][k]
    assert s["mustang_1_core"]["tron1"] == 225.0 and s["wolf_1_core"]["tron1"] == 98.4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
