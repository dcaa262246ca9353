"""bench.py host logic that needs no GPU: the one-GPU rule and the roofline
bookkeeping helpers."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_heff_flops_and_sampling_flops():
    import bench
    from paper_2210_03763_amd import workload as W
    w = W.config("c3")
    fps = bench.heff_flops_per_step(w)
    # 27.2 TFLOP of H_eff / K_eff matvecs per step at 8x8, d = 4, chi = 128
    assert 2.6e13 < fps < 2.9e13
    # per shot: two batch GEMMs (16 D_L D_R D_P real flops) per node above the bottom
    assert 4.0e8 < bench.sample_flops_per_shot(w) < 5.5e8


def test_traffic_summary_tracks_the_contraction_source(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter summary only while
    the contraction source still has the hash recorded there and the workload
    matches; otherwise it is null."""
    import bench
    src = tmp_path / "contract.hip"
    src.write_bytes(b"// kernel source\n")
    import hashlib
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "traffic.md"
    summary.write_text(f"- workload: W1\n- contract_source_sha256: `{sha}`\n- hbm_bytes_per_heff_launch: 123456\n")
    monkeypatch.setattr(bench, "CONTRACT_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench.measured_traffic("W1") == 123456.0
    assert bench.measured_traffic("W2") is None
    src.write_bytes(b"// kernel source, changed\n")
    assert bench.measured_traffic("W1") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic("W1") is None

