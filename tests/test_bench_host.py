"""Host-side logic of bench.py (no GPU): the one-GPU contract and the traffic record."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_is_keyed_to_the_kernel_sources(tmp_path, monkeypatch):
    """The committed counter summary carries the hash of the kernel sources it was taken with; the
    benchmark reports its traffic while that hash matches and null once the sources change."""
    import bench
    h = bench.hot_source_hash()
    assert len(h) == 64
    rec = tmp_path / "counters.txt"
    rec.write_text(f"traffic_bytes_per_call: 1234\nsource_sha256: {h}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.recorded_traffic() == 1234
    rec.write_text("traffic_bytes_per_call: 1234\nsource_sha256: " + "0" * 64 + "\n")
    assert bench.recorded_traffic() is None
    text = open(os.path.join(ROOT, "profiles", "k_loglike_moments_c2_hbm_counters.txt")).read()
    assert "traffic_bytes_per_call:" in text and "source_sha256:" in text
