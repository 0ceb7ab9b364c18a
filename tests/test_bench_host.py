"""Host logic of bench.py (no GPU): the one-GPU guard, the workload table,
the algorithmic byte counts and the rule that voids the committed HBM
traffic once the sweep kernels' sources change."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_cell():
    # 3D: 9 updated fields read and written, the increment-start pressure and
    # 5 stress components and the cohesion read (18 + 6 + 1); 2D: 6 read and
    # written, the increment-start pressure and 3 stresses and the cohesion
    # read (12 + 4 + 1)
    assert bench.bytes_per_cell(3, 4) == 100 and bench.bytes_per_cell(3, 8) == 200
    assert bench.bytes_per_cell(2, 4) == 68 and bench.bytes_per_cell(2, 8) == 136


def test_workload_table():
    m, desc = bench.workload("3d-511")
    assert (m.nx, m.ny, m.nz) == (511, 511, 511) and m.freeze_iter == 16 * 511
    assert "511" in desc
    m, _ = bench.workload("3d-255-het")
    assert m.nx == 255 and m.shear == pytest.approx(1.2)     # bounds the per-cell G (1 to 1.2)
    m, _ = bench.workload("2d-1023-het")
    assert (m.ndim, m.nx, m.ny) == (2, 1023, 1023) and m.freeze_iter == 16 * 1023
    with pytest.raises(SystemExit):
        bench.workload("4d-7")


def test_traffic_is_void_once_the_kernel_sources_change(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("3d-9", "fp32") is None           # no counters at all
    rec = {"hbm_bytes_per_sweep": 123456, "kernel_sources_sha256_16": "0123456789abcdef"}
    (prof / "traffic_3d-9_fp32.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0123456789abcdef")
    assert bench.measured_traffic("3d-9", "fp32") == 123456
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "fedcba9876543210")
    assert bench.measured_traffic("3d-9", "fp32") is None


def test_kernel_sources_hash_covers_the_sweep_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2305_01701_amd" / "csrc"
    csrc.mkdir(parents=True)
    names = ("ep_device.h", "ep_internal.h", "ep_sweep_fused.hip", "ep_sweep_unfused.hip")
    for f in names:
        (csrc / f).write_text(f"// {f}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sources_hash()
    for f in names:
        p = csrc / f
        old = p.read_text()
        p.write_text(old + " ")
        assert bench.kernel_sources_hash() != h0, f
        p.write_text(old)
    assert bench.kernel_sources_hash() == h0
