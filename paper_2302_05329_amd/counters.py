"""Summaries of rocprofv3 runs for the roofline figures (what the benchmark reports as measured
FP64 rates and HBM traffic), and the source hashes that tie a summary to the kernels it measured.

A summary is a short text file: a header with the commands that produced it, one row per kernel
(dispatches, average duration, calibrated HBM bytes and FP64 flops per dispatch of the last
call), then `key: value` lines that the benchmark reads:

    source_sha256: <hash of the sources the kernels are built from>
    <kernels label>_fp64_flops_per_call: N    (64 x (ADD + MUL + TRANS + 2 FMA) F64 instructions,
                                               plus 512 x SQ_INSTS_VALU_MFMA_MOPS_F64 when counted)
    <kernels label>_hbm_bytes_per_call: N     (calibrated FETCH_SIZE + WRITE_SIZE)

    python -m paper_2302_05329_amd.counters --title T --trace DIR [--fp64 DIR] [--fetch DIR
        --write DIR --cfetch DIR --cwrite DIR] --group loglike|mismatch --kernels LABEL=REGEX ...
        --command CMD ... --out FILE

DIR are rocprofv3 `-d` output folders (CSV format).  FETCH_SIZE and WRITE_SIZE are in KiB per
dispatch; each is scaled by what the same counter reads for a plain device-to-device copy of
known size (`bench.py --copy-calibration`, 1 GiB read and written).  Counts are those of the
last dispatch of each kernel name (the dispatches of one call of a deterministic pass).
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
GROUPS = {
    "loglike": ["pd_kernels.hip", "pd_bin.h", "pd_math.h", "pd_model.h", "pd_dual.h", "pd_launch.h"],
    "mismatch": ["pd_mismatch.hip", "pd_mismatch.h", "pd_bin.h", "pd_math.h", "pd_model.h", "pd_dual.h",
                 "pd_launch.h"],
    "overlap": ["pd_overlap.hip", "pd_bin.h", "pd_math.h", "pd_model.h", "pd_dual.h", "pd_launch.h"],
}
COPY_BYTES = 1 << 30
F64 = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64")


def source_hash(group):
    """sha256 over the sources of one kernel group."""
    h = hashlib.sha256()
    for name in GROUPS[group]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_summary(path, group):
    """The `key: value` lines of a summary, or None when it is missing or its source hash does not
    match the current sources of `group`."""
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    kv = {}
    for line in lines:
        if ":" in line and not line.startswith("#") and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash(group):
        return None
    return kv


def _csv(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            rows.extend(csv.DictReader(f))
    return rows


def counters_last(d):
    """{kernel name: {counter: value}} of the last dispatch of each kernel name."""
    by = collections.defaultdict(dict)
    for r in _csv(d, "counter_collection.csv"):
        disp = int(r["Dispatch_Id"])
        by[r["Kernel_Name"]].setdefault(disp, collections.Counter())[r["Counter_Name"]] += float(r["Counter_Value"])
    return {k: v[max(v)] for k, v in by.items()}


def durations(d):
    """{kernel name: (dispatches, average ns)} from a --kernel-trace run."""
    acc = collections.defaultdict(list)
    for r in _csv(d, "kernel_trace.csv"):
        acc[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def timeline(d, rx):
    """Start offset, duration (us) and name of every dispatch from one dispatch of the kernel
    matching `rx` to the next (the interval a quarter of the way through the trace)."""
    rows = sorted(_csv(d, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if re.search(rx, r["Kernel_Name"])]
    if len(marks) < 2:
        return ["# timeline: fewer than two dispatches of the marker kernel"]
    m = max(1, len(marks) // 4)
    i0, i1 = marks[m - 1], marks[m]
    t0 = int(rows[i0]["Start_Timestamp"])
    out = [f"timeline of one interval ({rx}), start_us duration_us kernel:"]
    for r in rows[i0:i1 + 1]:
        st = (int(r["Start_Timestamp"]) - t0) / 1e3
        du = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        out.append(f"  {st:9.1f} {du:8.1f}  {r['Kernel_Name'][:90]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--title", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fp64")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--cfetch")
    ap.add_argument("--cwrite")
    ap.add_argument("--group", required=True, choices=sorted(GROUPS))
    ap.add_argument("--kernels", nargs="+", required=True, help="LABEL=REGEX on the kernel name")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--note", action="append", default=[])
    ap.add_argument("--timeline", help="REGEX: list the dispatches between two consecutive dispatches of the "
                                       "matching kernel (a quarter of the way through the trace)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    labels = [kv.split("=", 1) for kv in a.kernels]
    dur = durations(a.trace)
    f64 = counters_last(a.fp64) if a.fp64 else {}
    hbm = None
    if a.fetch:
        fetch, write = counters_last(a.fetch), counters_last(a.write)
        cf = counters_last(a.cfetch)
        cw = counters_last(a.cwrite)
        copy = [k for k in cf if "copy" in k.lower()]
        kf = COPY_BYTES / 1024 / cf[copy[0]]["FETCH_SIZE"]
        kw = COPY_BYTES / 1024 / cw[copy[0]]["WRITE_SIZE"]
        hbm = (fetch, write, kf, kw)
    names = sorted(set(dur) | set(f64))
    out = [f"# {a.title}", "# commands (R = repository root on the GPU host):"]
    out += [f"#   {c}" for c in a.command]
    if hbm:
        out.append(f"# calibration: a plain 1 GiB device-to-device copy: FETCH_SIZE x {hbm[2]:.3f}, "
                   f"WRITE_SIZE x {hbm[3]:.3f}")
    out.append("")
    out.append(f"{'kernel':<44} {'calls':>6} {'avg_us':>9} {'hbm_bytes':>12} {'GB/s':>8} {'fp64_flops':>14} "
               f"{'TFLOP/s':>8} {'fp64_frac':>9}")
    totals = {}
    for label, rx in labels:
        tb, tf, tus = 0.0, 0.0, 0.0
        for k in names:
            if not re.search(rx, k):
                continue
            calls, ns = dur.get(k, (0, float("nan")))
            b = None
            if hbm and k in hbm[0]:
                b = hbm[0][k].get("FETCH_SIZE", 0) * 1024 * hbm[2] + hbm[1].get(k, {}).get("WRITE_SIZE", 0) * 1024 * hbm[3]
            fl = None
            if k in f64:
                c = f64[k]
                fl = 64 * (c["SQ_INSTS_VALU_ADD_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_TRANS_F64"]
                           + 2 * c["SQ_INSTS_VALU_FMA_F64"])
                # FP64 matrix-core work, when counted: the counter is in units of 512 flops
                fl += 512 * c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
            gbs = b / ns if b is not None and ns == ns else float("nan")
            tfs = fl / ns / 1e3 if fl is not None and ns == ns else float("nan")
            out.append(f"{k[:44]:<44} {calls:>6} {ns / 1e3:>9.2f} {(b or 0):>12.0f} {gbs:>8.1f} {(fl or 0):>14.0f} "
                       f"{tfs:>8.2f} {tfs / 78.6:>9.4f}")
            tb += b or 0.0
            tf += fl or 0.0
            tus += ns / 1e3 if ns == ns else 0.0
        totals[label] = (tb, tf, tus)
    out.append("")
    out.append(f"source_sha256: {source_hash(a.group)}")
    for label, (tb, tf, tus) in totals.items():
        if hbm:
            out.append(f"{label}_hbm_bytes_per_call: {int(round(tb))}")
        if f64:
            out.append(f"{label}_fp64_flops_per_call: {int(round(tf))}")
        out.append(f"{label}_avg_us_sum: {tus:.2f}")
    if a.timeline:
        out += [""] + timeline(a.trace, a.timeline)
    out += [f"# {n}" for n in a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


if __name__ == "__main__":
    main()
