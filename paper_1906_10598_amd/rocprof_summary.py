"""Summarise rocprofv3 output of one kernel into a short text file.

Reads the CSV directories written by

  rocprofv3 --kernel-trace --stats -d DIR/trace -o run --output-format csv -- python3 bench.py <mode>
  rocprofv3 --pmc FETCH_SIZE -d DIR/FETCH_SIZE -o run --output-format csv -- python3 bench.py <mode>
  rocprofv3 --pmc WRITE_SIZE -d DIR/WRITE_SIZE -o run --output-format csv -- python3 bench.py <mode>
  rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES SQ_BUSY_CYCLES GRBM_GUI_ACTIVE -d DIR/SQ_INSTS_VALU ...
  rocprofv3 --pmc SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_TRANS_F64
                  SQ_INSTS_VALU_FMA_F32 SQ_INSTS_VALU_ADD_F32 SQ_INSTS_VALU_MUL_F32 SQ_INSTS_VALU_TRANS_F32
                  -d DIR/SQ_INSTS_VALU_FMA_F64 ...

and writes a markdown summary: the per-kernel average duration, the
counters per dispatch of the kernel named (median over its dispatches), the
HBM traffic (FETCH_SIZE / WRITE_SIZE scaled by what the same counters read
for a calibration elementwise kernel of known size: 256 MiB read, 256 MiB
written), the executed FP64 / FP32 operations and the VALU issue fraction.
Two machine-readable lines carry the figures bench.py reports:

  traffic: bytes_per_launch=... kernel_hash=... workload=... geometry=S,C form=...
  counters: kernel_hash=... workload=... geometry=S,C form=... avg_us=... valu=... fma_f64=... ...

bench.py uses them only while the kernel sources still hash to kernel_hash.

Usage: python -m paper_1906_10598_amd.rocprof_summary DIR OUT.md KERNEL_SUBSTRING "COMMAND TEXT" FORM WORKLOAD
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
CSRC = os.path.join(ROOT, "paper_1906_10598_amd", "csrc")
# every source a kernel's code or launch depends on
KERNEL_SOURCES = ("kernels.h", "device.h", "cospoly.h", "instances.h", "instances.hip", "phasetrack.hip")
CAL_BYTES = 256 * 1024 * 1024
# counters whose per-dispatch medians go on the `counters:` line
COUNTER_KEYS = {"SQ_INSTS_VALU": "valu", "SQ_WAVES": "waves",
                "SQ_INSTS_VALU_FMA_F64": "fma_f64", "SQ_INSTS_VALU_ADD_F64": "add_f64",
                "SQ_INSTS_VALU_MUL_F64": "mul_f64", "SQ_INSTS_VALU_TRANS_F64": "trans_f64",
                "SQ_INSTS_VALU_FMA_F32": "fma_f32", "SQ_INSTS_VALU_ADD_F32": "add_f32",
                "SQ_INSTS_VALU_MUL_F32": "mul_f32", "SQ_INSTS_VALU_TRANS_F32": "trans_f32"}


def kernel_hash():
    """sha256 of the kernel sources and of build.py (its compiler flags shape
    the code too), first 16 hex digits."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_1906_10598_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def executed_flop(c):
    """FP64 and FP32 operations per dispatch from wave-instruction counters:
    64 lanes per wave64 instruction, two operations per FMA."""
    f64 = 64 * (2 * c.get("fma_f64", 0) + c.get("add_f64", 0) + c.get("mul_f64", 0) + c.get("trans_f64", 0))
    f32 = 64 * (2 * c.get("fma_f32", 0) + c.get("add_f32", 0) + c.get("mul_f32", 0) + c.get("trans_f32", 0))
    return f64, f32


def read_profile(path, workload, geometry, form):
    """The `traffic:` and `counters:` figures of a committed summary, if it was
    taken with the current kernel sources, workload, geometry and form."""
    out = {}
    try:
        with open(path) as f:
            for line in f:
                tag = line.split(":", 1)[0]
                if tag not in ("traffic", "counters"):
                    continue
                kv = dict(item.split("=", 1) for item in line.split()[1:])
                if (kv.get("kernel_hash") == kernel_hash() and kv.get("workload") == workload
                        and kv.get("geometry") == "%d,%d" % tuple(geometry) and kv.get("form") == form):
                    for k, v in kv.items():
                        if k not in ("kernel_hash", "workload", "geometry", "form"):
                            out[k] = float(v)
    except (OSError, ValueError, KeyError):
        return {}
    return out


def _counters(path):
    d = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return d


def summarise(root, kernel, command, form, workload):
    out = []
    stats = os.path.join(root, "trace", "run_kernel_stats.csv")
    avg_ns = calls = None
    out.append("## Kernel trace (rocprofv3 --kernel-trace --stats)\n")
    out.append("| kernel | calls | average [us] | min [us] | max [us] |")
    out.append("|---|---|---|---|---|")
    for r in csv.DictReader(open(stats)):
        name = r["Name"]
        out.append(f"| `{name[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
        if kernel in name and avg_ns is None:
            avg_ns, calls = float(r["AverageNs"]), int(r["Calls"])
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
    out.append("| counter | kernel | calibration kernel (256 MiB in, 256 MiB out) |")
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
    cvals = {}
    if kern:
        cvals = {short: per[kern][c] for c, short in COUNTER_KEYS.items() if c in per[kern]}
    if "valu" in cvals and avg_ns:
        cap = 1024 * avg_ns * 1e-9 * 2.4e9 / 4.0
        out.append(f"VALU issue: {cvals['valu']:.4g} wave64 instructions per launch; at one wave64 "
                   f"instruction per 4 cycles per SIMD, 1024 SIMDs and 2.4 GHz the launch could issue "
                   f"{cap:.4g}: {cvals['valu'] / cap:.1%} of the issue slots.\n")
    if "fma_f64" in cvals and avg_ns:
        f64, f32 = executed_flop(cvals)
        out.append(f"Executed operations per launch (counters x 64 lanes, FMA x 2): FP64 {f64:.4g}, FP32 {f32:.4g}; "
                   f"at the average duration: FP64 {f64 / (avg_ns * 1e-9) / 1e12:.2f} TFLOP/s "
                   f"({f64 / (avg_ns * 1e-9) / 78.6e12:.1%} of 78.6), FP32 {f32 / (avg_ns * 1e-9) / 1e12:.2f} TFLOP/s.\n")
    geo = ""
    m = re.search(r"k_objective<\w+, (\d+), (\d+)", kernel)
    if m:
        geo = f" geometry={m.group(1)},{m.group(2)}"
    head = [f"# rocprofv3 summary: `{kernel}`\n", "Command(s):\n", "```", command, "```\n",
            f"Kernel sources hash: {kernel_hash()} (sha256 of csrc/{', '.join(KERNEL_SOURCES)} and build.py)\n"]
    if avg_ns:
        head.append(f"Average duration of the kernel: {avg_ns / 1e3:.3f} us over {calls} dispatches\n")
    if traffic is not None:
        head.append(f"traffic: bytes_per_launch={traffic:.0f} kernel_hash={kernel_hash()} "
                    f"workload={workload}{geo} form={form}\n")
    if cvals:
        kv = " ".join(f"{k}={v:.6g}" for k, v in sorted(cvals.items()))
        head.append(f"counters: kernel_hash={kernel_hash()} workload={workload}{geo} form={form} "
                    f"avg_us={(avg_ns or 0) / 1e3:.4f} {kv}\n")
    return "\n".join(head + out) + "\n"


def main():
    root, out_path, kernel, command, form, workload = sys.argv[1:7]
    text = summarise(root, kernel, command, form, workload)
    with open(out_path, "w") as fh:
        fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
