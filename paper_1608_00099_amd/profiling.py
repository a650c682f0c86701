"""Summaries of rocprofv3 output for profiles/ (kernel statistics and HBM
traffic), and the traffic record bench.py reads.

Usage (after the rocprofv3 runs whose commands the summaries quote):
  python -m paper_1608_00099_amd.profiling stats STATS_CSV OUT_MD "COMMAND"
  python -m paper_1608_00099_amd.profiling traffic FETCH_DIR WRITE_DIR KERNEL OUT_JSON OUT_MD "COMMANDS"

Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) come from two
separate counter runs of the same command (`-o sweep`), each calibrated by
what the same counter reads for a plain device copy of 1 GiB (`-o ceil`,
torch's copy kernel): calibrated bytes = counter KiB * 1024 * (2^30 /
counter reading of the 1 GiB copy).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GIB = 1 << 30


def kernel_source_hash():
    """Hash of the kernel and planner sources (a traffic record is valid
    only for the sources it was measured on)."""
    h = hashlib.sha256()
    for f in ("common.h", "kern_coiter.hip", "kern_segment.hip", "kern_reduce.hip", "plan.cpp"):
        with open(os.path.join(ROOT, "paper_1608_00099_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def stats_markdown(stats_csv, command):
    rows = _rows(stats_csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["Command: `%s`" % command, "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        name = r["Name"] if len(r["Name"]) <= 160 else r["Name"][:157] + "..."
        out.append("| `%s` | %s | %.2f | %.2f | %.2f | %.2f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def _per_kernel(path, counter):
    agg = {}
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        agg.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return agg


def _calibration(ceil_csv, counter):
    agg = _per_kernel(ceil_csv, counter)
    vals = [v for k, vs in agg.items() if "copyBuffer" in k or "copy" in k.lower() for v in vs]
    vals = [v for v in vals if v > 1e5]
    if not vals:
        raise SystemExit("no 1 GiB copy dispatch found in %s" % ceil_csv)
    kib = sorted(vals)[len(vals) // 2]
    return GIB / (kib * 1024.0), kib


def traffic(fetch_dir, write_dir, kernel):
    ff, fk = _calibration(os.path.join(fetch_dir, "ceil_counter_collection.csv"), "FETCH_SIZE")
    wf, wk = _calibration(os.path.join(write_dir, "ceil_counter_collection.csv"), "WRITE_SIZE")
    fetch = _per_kernel(os.path.join(fetch_dir, "sweep_counter_collection.csv"), "FETCH_SIZE")
    write = _per_kernel(os.path.join(write_dir, "sweep_counter_collection.csv"), "WRITE_SIZE")
    if kernel not in fetch or kernel not in write:
        raise SystemExit("kernel %r not in the counter runs" % kernel)
    f = sum(fetch[kernel]) / len(fetch[kernel]) * 1024.0 * ff
    w = sum(write[kernel]) / len(write[kernel]) * 1024.0 * wf
    return {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w,
            "bytes_per_launch": f + w, "dispatches": len(fetch[kernel]),
            "fetch_calibration": ff, "write_calibration": wf,
            "copy_1GiB_fetch_kib": fk, "copy_1GiB_write_kib": wk,
            "source_hash": kernel_source_hash()}


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        md = stats_markdown(argv[1], argv[3])
        with open(argv[2], "w") as f:
            f.write(md)
        return 0
    if len(argv) >= 7 and argv[0] == "traffic":
        fetch_dir, write_dir, kernel, out_json, out_md, commands = argv[1:7]
        rec = traffic(fetch_dir, write_dir, kernel)
        table = {}
        if os.path.exists(out_json):
            with open(out_json) as f:
                table = json.load(f)
        table[kernel] = rec
        with open(out_json, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        with open(out_md, "w") as f:
            f.write("Commands: `%s`\n\n" % commands)
            f.write("Kernel: `%s`\n\n" % kernel)
            f.write("| quantity | value |\n|---|---:|\n")
            for k in ("fetch_bytes_per_launch", "write_bytes_per_launch", "bytes_per_launch",
                      "dispatches", "fetch_calibration", "write_calibration",
                      "copy_1GiB_fetch_kib", "copy_1GiB_write_kib"):
                f.write("| %s | %s |\n" % (k, rec[k]))
            f.write("| source_hash | %s |\n" % rec["source_hash"])
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
