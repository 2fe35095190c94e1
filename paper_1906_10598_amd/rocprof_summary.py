"""Summarise rocprofv3 output of the objective kernel into a short text file.

Reads the CSV directories written by

  rocprofv3 --kernel-trace --stats -d DIR/trace -o run --output-format csv -- python3 bench.py --kernel-only ...
  rocprofv3 --pmc FETCH_SIZE -d DIR/FETCH_SIZE -o run --output-format csv -- python3 bench.py --kernel-only ...
  rocprofv3 --pmc WRITE_SIZE -d DIR/WRITE_SIZE -o run --output-format csv -- ...
  (optional) further --pmc passes, one directory each

and writes a markdown summary with the per-kernel average duration, the
traffic counters per dispatch (scaled by the calibration elementwise kernel
of known size: 256 MiB read, 256 MiB written) and the VALU counters.  The
summary carries a `traffic:` line that bench.py reads (bytes per launch and
the hash of the kernel sources they were taken with).

Usage: python -m paper_1906_10598_amd.rocprof_summary DIR OUT.md KERNEL_SUBSTRING "COMMAND TEXT" [FORM]

FORM names the launch form the counters were taken in: "objective" (default,
bench.py --kernel-only: the objective alone) or "fit-lead" (bench.py
--fit-only: the fit's launches with the leading DE step).
"""
import csv
import glob
import hashlib
import os
import re
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CAL_BYTES = 256 * 1024 * 1024


def kernel_hash():
    h = hashlib.sha256()
    for f in ("kernels.h", "device.h"):
        with open(os.path.join(ROOT, "paper_1906_10598_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counters(path):
    d = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return d


def summarise(root, kernel, command, form="objective"):
    out = []
    stats = os.path.join(root, "trace", "run_kernel_stats.csv")
    avg_ns = None
    out.append("## Kernel trace (rocprofv3 --kernel-trace --stats)\n")
    out.append("| kernel | calls | average [us] | min [us] | max [us] |")
    out.append("|---|---|---|---|---|")
    for r in csv.DictReader(open(stats)):
        name = r["Name"]
        out.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
        if kernel in name and avg_ns is None:
            avg_ns = float(r["AverageNs"])
    out.append("")
    per = {}
    for d in sorted(glob.glob(os.path.join(root, "*", "run_counter_collection.csv"))):
        for kname, ctrs in _counters(d).items():
            for c, vals in ctrs.items():
                per.setdefault(kname, {})[c] = statistics.median(vals)
    kern = next((k for k in per if kernel in k), None)
    cal = next((k for k in per if "elementwise" in k and "WRITE_SIZE" in per[k] and per[k].get("WRITE_SIZE", 0) > 1e5
                and "FillFunc" not in k), None)
    fetch_scale = write_scale = None
    if cal:
        if per[cal].get("FETCH_SIZE"):
            fetch_scale = CAL_BYTES / (per[cal]["FETCH_SIZE"] * 1024)
        if per[cal].get("WRITE_SIZE"):
            write_scale = CAL_BYTES / (per[cal]["WRITE_SIZE"] * 1024)
    out.append("## Counters per dispatch (median over dispatches; rocprofv3 --pmc, one pass per group)\n")
    out.append("| counter | objective kernel | calibration kernel (256 MiB in, 256 MiB out) |")
    out.append("|---|---|---|")
    if kern:
        for c in sorted(per[kern]):
            calv = per[cal].get(c, "") if cal else ""
            out.append(f"| {c} | {per[kern][c]:.6g} | {calv if calv == '' else f'{calv:.6g}'} |")
    out.append("")
    traffic = None
    if kern and "FETCH_SIZE" in per[kern] and "WRITE_SIZE" in per[kern]:
        fb = per[kern]["FETCH_SIZE"] * 1024 * (fetch_scale or 1.0)
        wb = per[kern]["WRITE_SIZE"] * 1024 * (write_scale or 1.0)
        traffic = fb + wb
        out.append(f"HBM traffic per launch: fetch {fb / 1e6:.3f} MB + write {wb / 1e6:.3f} MB "
                   f"= {traffic / 1e6:.3f} MB (counter KiB x 1024 x calibration factor; factors "
                   f"fetch {fetch_scale}, write {write_scale}).\n")
    if kern and "SQ_INSTS_VALU" in per[kern] and avg_ns:
        wave_instr = per[kern]["SQ_INSTS_VALU"]
        cap = 1024 * avg_ns * 1e-9 * 2.4e9 / 4.0
        out.append(f"VALU issue: {wave_instr:.4g} wave64 instructions per launch; at one wave64 "
                   f"instruction per 4 cycles per SIMD, 1024 SIMDs and 2.4 GHz the launch could issue "
                   f"{cap:.4g}: {wave_instr / cap:.1%} of the issue slots.\n")
    head = [f"# rocprofv3 summary: `{kernel}`\n", "Command(s):\n", "```", command, "```\n",
            f"Kernel sources hash: {kernel_hash()}\n"]
    if avg_ns:
        head.append(f"Average duration of the kernel: {avg_ns / 1e3:.3f} us\n")
    if traffic is not None:
        geo = ""
        m = re.search(r"k_objective<\w+, (\d+), (\d+)", kernel)
        if m:
            geo = f" geometry={m.group(1)},{m.group(2)}"
        head.append(f"traffic: bytes_per_launch={traffic:.0f} kernel_hash={kernel_hash()} "
                    f"workload=paper-400000-fp32{geo} form={form}\n")
    return "\n".join(head + out) + "\n"


def main():
    root, out_path, kernel, command = sys.argv[1:5]
    form = sys.argv[5] if len(sys.argv) > 5 else "objective"
    text = summarise(root, kernel, command, form)
    with open(out_path, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
