"""Host logic of bench.py, no GPU: the algorithmic byte count of one MTTKRP,
the recorded-traffic lookup (used only while it describes the built kernel
sources), and the one-GPU guard."""

import json
import os
import subprocess
import sys

import bench


def test_algorithmic_bytes():
    # 512^3 FP32, R=32: X at 4 B per element, the two input factors, the output.
    assert bench.algorithmic_bytes((512, 512, 512), 32, 0, "fp32") == 512**3 * 4 + 4 * 32 * 1024 + 4 * 512 * 32
    # FP8 768^3, R=128, mode index 1: 1 B per element plus one exponent per
    # mode-1 slice.
    assert bench.algorithmic_bytes((768, 768, 768), 128, 1, "fp8") == 768**3 + 4 * 128 * 1536 + 4 * 768 * 128 + 4 * 768
    # Skewed shape: the input factors are those of the other two modes.
    assert bench.algorithmic_bytes((10, 20, 30), 8, 2, "fp32") == 6000 * 4 + 4 * 8 * 30 + 4 * 30 * 8


def test_recorded_traffic_follows_kernel_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"workload": "w", "prec": "fp32", "kernel_sources_sha256_16": "abcd" * 4,
           "traffic_bytes_per_launch_mean": 123.0}
    (tmp_path / "profiles" / "traffic_w_fp32.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "abcd" * 4)
    assert bench.recorded_traffic("w", "fp32") == 123.0
    assert bench.recorded_traffic("w", "bf16x3") is None          # no record for it
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0" * 16)
    assert bench.recorded_traffic("w", "fp32") is None            # sources changed since


def test_kernel_sources_hash_is_stable():
    h = bench.kernel_sources_hash()
    assert len(h) == 16 and h == bench.kernel_sources_hash()


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_kernel_source_files_cover_the_dense_kernels_only():
    files = bench.kernel_source_files()
    assert "mttkrp_kernels.hip" in files and "dimtree.hip" in files and "tile_device.h" in files
    assert not {"sparse.hip", "server.hip", "als_kernels.hip", "api.hip"} & set(files)


def test_recorded_traffic_per_kernel(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"workload": "w", "prec": "fp8", "kernel_sources_sha256_16": "abcd" * 4,
           "traffic_bytes_per_launch": {"k1": 10.0, "k2": 20.0}}
    (tmp_path / "profiles" / "traffic_w_fp8.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "abcd" * 4)
    assert bench.recorded_traffic("w", "fp8", "k2") == 20.0
    assert bench.recorded_traffic("w", "fp8", "k3") is None
    assert bench.recorded_traffic("w", "fp8") is None
