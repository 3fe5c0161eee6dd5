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
    for path, group, label in ((bench.COUNTERS_C1, "loglike", "waveform"), (bench.COUNTERS_C3, "loglike", "fisher"),
                               (bench.COUNTERS_OV, "overlap", "gemm")):
        kv = counters.read_summary(path, group)
        assert kv is not None, f"{os.path.basename(path)} is stale"
        assert int(kv[f"{label}_fp64_flops_per_call"]) > 0 and int(kv[f"{label}_hbm_bytes_per_call"]) > 0


def test_counter_summary_from_synthetic_profiler_output(tmp_path, monkeypatch):
    """counters.py on tiny hand-written rocprofv3-style CSVs: per-kernel averages, the last
    dispatch's FP64 flops (64 x (ADD + MUL + TRANS + 2 FMA)), bytes scaled by the copy calibration,
    the summed keys and the timeline between two dispatches of a marker kernel."""
    import csv as _csv
    from paper_2302_05329_amd import counters

    def write(d, name, rows):
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name), "w", newline="") as f:
            w = _csv.DictWriter(f, fieldnames=list(rows[0].keys()))
            w.writeheader()
            w.writerows(rows)

    tr = tmp_path / "trace"
    write(tr, "run_kernel_trace.csv", [
        {"Kernel_Name": "k_begin", "Start_Timestamp": 0, "End_Timestamp": 1000},
        {"Kernel_Name": "k_a", "Start_Timestamp": 2000, "End_Timestamp": 6000},
        {"Kernel_Name": "k_begin", "Start_Timestamp": 7000, "End_Timestamp": 8000},
        {"Kernel_Name": "k_a", "Start_Timestamp": 9000, "End_Timestamp": 11000}])
    f64 = tmp_path / "f64"
    rows = []
    for disp, scale in ((1, 1), (2, 2)):
        for c, v in (("SQ_INSTS_VALU_ADD_F64", 10), ("SQ_INSTS_VALU_MUL_F64", 20), ("SQ_INSTS_VALU_FMA_F64", 30),
                     ("SQ_INSTS_VALU_TRANS_F64", 5)):
            rows.append({"Dispatch_Id": disp, "Kernel_Name": "k_a", "Counter_Name": c, "Counter_Value": v * scale})
    write(f64, "run_counter_collection.csv", rows)
    fe, wr, cf, cw = (tmp_path / n for n in ("fe", "wr", "cf", "cw"))
    write(fe, "run_counter_collection.csv", [{"Dispatch_Id": 2, "Kernel_Name": "k_a", "Counter_Name": "FETCH_SIZE", "Counter_Value": 100}])
    write(wr, "run_counter_collection.csv", [{"Dispatch_Id": 2, "Kernel_Name": "k_a", "Counter_Name": "WRITE_SIZE", "Counter_Value": 50}])
    write(cf, "run_counter_collection.csv", [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288}])
    write(cw, "run_counter_collection.csv", [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576}])
    out = tmp_path / "s.txt"
    monkeypatch.setattr(sys, "argv", ["counters", "--title", "t", "--trace", str(tr), "--fp64", str(f64), "--fetch", str(fe), "--write", str(wr),
                "--cfetch", str(cf), "--cwrite", str(cw), "--group", "loglike", "--kernels", "a=k_a",
                "--timeline", "k_begin", "--out", str(out)])
    counters.main()
    kv = counters.read_summary(str(out), "loglike")
    # last dispatch: 64 x (20 + 40 + 10 + 2 x 60) = 12160 flops; bytes: 100 KiB x 2 + 50 KiB x 1
    assert int(kv["a_fp64_flops_per_call"]) == 64 * (20 + 40 + 10 + 2 * 60)
    assert int(kv["a_hbm_bytes_per_call"]) == 100 * 1024 * 2 + 50 * 1024
    assert abs(float(kv["a_avg_us_sum"]) - 3.0) < 1e-9
    text = out.read_text()
    assert "timeline of one interval" in text and "k_a" in text.split("timeline")[1]
