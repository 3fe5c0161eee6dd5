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


def test_counter_summary_is_keyed_to_the_kernel_sources(tmp_path):
    """A counter summary carries the hash of the kernel sources it was taken with; it is read while
    that hash matches and ignored once the sources change (the benchmark then reports the
    algorithmic rate and a null traffic)."""
    from paper_2302_05329_amd import counters
    h = counters.source_hash("loglike")
    assert len(h) == 64 and h != counters.source_hash("mismatch")
    rec = tmp_path / "counters.txt"
    rec.write_text(f"# title\nmoments_fp64_flops_per_call: 1234\nsource_sha256: {h}\n")
    assert counters.read_summary(str(rec), "loglike")["moments_fp64_flops_per_call"] == "1234"
    assert counters.read_summary(str(rec), "mismatch") is None
    rec.write_text("moments_fp64_flops_per_call: 1234\nsource_sha256: " + "0" * 64 + "\n")
    assert counters.read_summary(str(rec), "loglike") is None


def test_committed_summaries_match_the_current_kernels():
    """The summaries the benchmark reads were taken with the kernels as committed."""
    import bench
    from paper_2302_05329_amd import counters
    kv = counters.read_summary(bench.COUNTERS_C2, "loglike")
    assert kv is not None, "C2 counter summary is stale"
    assert int(kv["moments_fp64_flops_per_call"]) > 0 and int(kv["moments_hbm_bytes_per_call"]) > 0
    kv = counters.read_summary(bench.COUNTERS_C4, "mismatch")
    assert kv is not None, "C4 counter summary is stale"
    for key in ("columns_hbm_bytes_per_call", "rows_hbm_bytes_per_call", "adjoint_fp64_flops_per_call"):
        assert int(kv[key]) > 0
