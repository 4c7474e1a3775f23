"""The benchmark's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1",
                        "--warmup", "0"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_is_used_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    """`roofline.traffic` comes from a committed counter summary only while the
    kernel sources still hash to the value recorded with it."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    rec = {"kernel_source_sha256_16": bench.kernel_source_hash(),
           "kernels": {"k_sobolev": {"bytes_per_launch": 123.0}}}
    (tmp_path / "hbm_traffic_w.md").write_text("summary\n\n```json\n" + json.dumps(rec) + "\n```\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic("w", "k_sobolev") == 123.0
    assert bench.measured_traffic("w", "k_flip") is None       # kernel not in the record
    assert bench.measured_traffic("other", "k_sobolev") is None  # no summary for the workload
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "f" * 16)
    assert bench.measured_traffic("w", "k_sobolev") is None    # sources changed since
