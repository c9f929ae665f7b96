"""The measurement script's contract, checked on the host: one GPU only, and the
stored HBM traffic is reported only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_needs_matching_sources_and_kernel(tmp_path, monkeypatch):
    import bench
    path = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_JSON", str(path))
    rec = {"kernel_key": "stage2d_list_kernel<5", "kernel_sources_sha256": bench.stage_sources_hash(),
           "traffic_bytes_per_launch": 1.25e9}
    path.write_text(json.dumps(rec))
    assert bench.stored_traffic("stage2d_list_kernel<5") == 1.25e9
    assert bench.stored_traffic("stage2d_kernel<5") is None          # taken on the other stage kernel
    rec["kernel_sources_sha256"] = "0" * 64                           # kernel sources changed since
    path.write_text(json.dumps(rec))
    assert bench.stored_traffic("stage2d_list_kernel<5") is None
    path.write_text("not json")
    assert bench.stored_traffic("stage2d_list_kernel<5") is None
