"""Summaries of rocprofv3 output for profiles/ (kernel statistics and HBM
traffic), and the traffic record bench.py reads.

Usage (after the rocprofv3 runs whose commands the summaries quote):
  python -m paper_1608_00099_amd.profiling stats STATS_CSV OUT_MD "COMMAND"
  python -m paper_1608_00099_amd.profiling traffic FETCH_DIR WRITE_DIR KERNEL OUT_JSON OUT_MD "COMMANDS"
  python -m paper_1608_00099_amd.profiling counters BENCH_JSON OUT_MD "COMMANDS" PMC_DIR...

Counters: per launch of the d = 2..8 sweep (the co-iteration dispatches of
`bench.py --no-cpu --no-extras`, 14 per step in launch order, averaged over
the steps), the L2-to-memory request counts of one or more counter runs:
write requests and their 64-byte share (bytes = 32 per request + 32 per
64-byte request), read requests by size, DRAM credit stalls, and the
per-launch time and algorithmic bytes from the same command's bench line.

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
           "Kernel source: `%s` (paper_1608_00099_amd.profiling.kernel_source_hash)"
           % kernel_source_hash(), "",
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


SWEEP_LAUNCHES = [n for d in range(2, 9) for n in ("copy d=%d" % d, "mul_acc d=%d" % d)]


def sweep_counters(pmc_dirs):
    """{launch name: {counter: mean value per dispatch}} over the sweep's
    co-iteration dispatches of every counter run in pmc_dirs."""
    out = {n: {} for n in SWEEP_LAUNCHES}
    for d in pmc_dirs:
        files = [f for f in sorted(os.listdir(d)) if f.endswith("counter_collection.csv")]
        if not files:
            raise SystemExit("no counter_collection.csv in %s" % d)
        disp = {}
        for r in _rows(os.path.join(d, files[0])):
            if "coiter_kernel" not in r["Kernel_Name"]:
                continue
            disp.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        ids = sorted(disp)
        if not ids or len(ids) % len(SWEEP_LAUNCHES):
            raise SystemExit("%s: %d sweep dispatches, not whole steps" % (d, len(ids)))
        acc = {}
        for k, i in enumerate(ids):
            name = SWEEP_LAUNCHES[k % len(SWEEP_LAUNCHES)]
            for c, v in disp[i].items():
                acc.setdefault((name, c), []).append(v)
        for (name, c), vs in acc.items():
            out[name][c] = sum(vs) / len(vs)
    return out


def counters_markdown(bench_line, pmc_dirs, commands):
    per_op = bench_line["per_op"]
    cnt = sweep_counters(pmc_dirs)
    out = ["Commands: `%s`" % commands, "",
           "Kernel source: `%s` (paper_1608_00099_amd.profiling.kernel_source_hash)"
           % kernel_source_hash(), "",
           "Per launch of the sweep, averaged over the profiled steps.  alg: the algorithmic "
           "bytes (read and written).  Written bytes from the L2-to-memory write requests "
           "(32 B each, 64 B for the 64-byte ones); read bytes from the read requests by size "
           "(32, 64 and 128 B).  Stall columns count cycles summed over the L2 channels.", "",
           "| launch | ms | alg read MB | read MB | read/alg | alg write MB | write MB | "
           "write/alg | 64-B writes | DRAM write-credit stall | DRAM read-credit stall |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for name in SWEEP_LAUNCHES:
        c = cnt[name]
        op = per_op[name]
        alg = float(op["bytes"])
        alg_w = alg / 2 if name.startswith("copy") else alg / 4
        alg_r = alg - alg_w
        wr = c.get("TCC_EA0_WRREQ_sum")
        w64 = c.get("TCC_EA0_WRREQ_64B_sum")
        wbytes = (wr + w64) * 32 if wr is not None and w64 is not None else None
        rd = c.get("TCC_EA0_RDREQ_sum")
        r32 = c.get("TCC_EA0_RDREQ_32B_sum", 0.0)
        r64 = c.get("TCC_EA0_RDREQ_64B_sum")
        r128 = c.get("TCC_EA0_RDREQ_128B_sum")
        rbytes = (32 * r32 + 64 * r64 + 128 * r128) if (r64 is not None and r128 is not None) else None
        f = lambda v, k=1e6, p="%.1f": (p % (v / k)) if v is not None else "-"
        out.append("| %s | %.4f | %.1f | %s | %s | %.1f | %s | %s | %s | %s | %s |" % (
            name, op["ms"], alg_r / 1e6, f(rbytes), f(rbytes, alg_r, "%.3f") if rbytes else "-",
            alg_w / 1e6, f(wbytes), f(wbytes, alg_w, "%.3f") if wbytes else "-",
            ("%.1f%%" % (100.0 * w64 / wr)) if wr else "-",
            f(c.get("TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum"), 1, "%.0f"),
            f(c.get("TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum"), 1, "%.0f")))
    return "\n".join(out) + "\n"


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
    if len(argv) >= 5 and argv[0] == "counters":
        with open(argv[1]) as f:
            line = json.loads([ln for ln in f.read().splitlines() if ln.startswith("{")][-1])
        md = counters_markdown(line, argv[4:], argv[3])
        with open(argv[2], "w") as f:
            f.write(md)
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
