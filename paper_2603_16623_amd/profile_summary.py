"""Summaries of rocprofv3 output for the march kernel (markdown, a few KB).

    python -m paper_2603_16623_amd.profile_summary trace DIR TITLE COMMAND [KERNEL] > summary.md
    python -m paper_2603_16623_amd.profile_summary traffic MARCH_DIR COPY_DIR COPY_MIB WORKLOAD [KERNEL] > traffic.txt
    python -m paper_2603_16623_amd.profile_summary sq DIR RING_SLICES > sq.txt

KERNEL is the marcher whose dispatches are summarised: wake_march_kernel (the
default; one species over immobile ions) or ions_march_kernel (electrons and
mobile ions).

`trace`: DIR holds the CSV files of `rocprofv3 --kernel-trace --stats --output-format csv`;
prints the march dispatches and the top kernels.
`traffic`: MARCH_DIR / COPY_DIR hold `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs
(subfolders FETCH_SIZE/ and WRITE_SIZE/) of the profiling driver and of a plain copy of COPY_MIB
MiB; prints HBM bytes per march dispatch, each counter scaled by copy bytes / counter reading
of the copy, and the digest of the marcher sources the counters belong to.
`sq`: DIR holds `--pmc` runs of SQ counters (any subfolders) over march dispatches covering
RING_SLICES ring-slices in all; prints the counters summed over those dispatches, per
ring-slice, and the occupancy / issue ratios (SQ_WAVE_CYCLES and SQ_ACTIVE_INST_* count
four-cycle units, SQ_BUSY_CYCLES single cycles).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
MARCH_SOURCES = ["wake_march.hip", "wake_device.h", "wake_common.h", "wake_cluster.h", "wake_ring.h"]
ION_SOURCES = ["wake_ions.hip", "wake_ions.h", "wake_ring.h", "wake_device.h", "wake_common.h"]
SOURCES = {"wake_march_kernel": MARCH_SOURCES, "ions_march_kernel": ION_SOURCES}


def source_digest(kernel: str = "wake_march_kernel") -> str:
    h = hashlib.sha256()
    for f in SOURCES[kernel]:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(pattern):
    out = []
    for f in sorted(glob.glob(pattern, recursive=True)):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def trace(d, title, command, per_dispatch=True, kernel="wake_march_kernel"):
    trace_rows = _rows(os.path.join(d, "**", "*kernel_trace.csv")) if per_dispatch else []
    stats = _rows(os.path.join(d, "**", "*kernel_stats.csv"))
    print(f"# {title}\n\nCommand (repository root as $R):\n\n    {command}\n")
    march = [r for r in trace_rows if kernel in r.get("Kernel_Name", "")]
    if march:
        print("March dispatches in order:\n")
        print("| dispatch | variant | duration ms | grid threads | workgroup | arch VGPR | acc VGPR | SGPR | LDS B | scratch B |")
        print("|---|---|---|---|---|---|---|---|---|---|")
        for r in march:
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            name = r.get("Kernel_Name", "")
            var = name[name.find("<") + 1:name.find(">")] if "<" in name else ""
            print(f"| {r.get('Dispatch_Id', '')} | {var} | {dur:.3f} | {r.get('Grid_Size_X', r.get('Grid_Size', ''))} | "
                  f"{r.get('Workgroup_Size_X', r.get('Workgroup_Size', ''))} | {r.get('VGPR_Count', '')} | "
                  f"{r.get('Accum_VGPR_Count', '')} | {r.get('SGPR_Count', '')} | {r.get('LDS_Block_Size', '')} | "
                  f"{r.get('Scratch_Size', '')} |")
        print()
    if stats:
        print("Kernels by total time:\n")
        print("| kernel | calls | avg ms | min ms | max ms | total ms |")
        print("|---|---|---|---|---|---|")
        stats.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
        for r in stats[:12]:
            name = r["Name"][:90]
            print(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                  f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | "
                  f"{float(r['TotalDurationNs']) / 1e6:.2f} |")


def _counter(d, name, kernel_sub):
    vals = []
    for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
        if r["Counter_Name"] == name and kernel_sub in r["Kernel_Name"]:
            vals.append(float(r["Counter_Value"]))
    return vals


def traffic(march_dir, copy_dir, copy_mib, workload, kernel="wake_march_kernel"):
    copy_bytes = float(copy_mib) * (1 << 20)
    out = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = _counter(os.path.join(copy_dir, c), c, "copyBuffer")
        m = _counter(os.path.join(march_dir, c), c, kernel)
        scale = copy_bytes / (cal[-1] * 1024.0)
        out[c] = (m[-1] * 1024.0 * scale, scale, m[-1])
    print(f"workload: {workload}")
    print(f"kernel: {kernel}")
    print(f"source_digest: {source_digest(kernel)}")
    print(f"fetch_bytes_per_dispatch: {out['FETCH_SIZE'][0]:.6e}")
    print(f"write_bytes_per_dispatch: {out['WRITE_SIZE'][0]:.6e}")
    print(f"fetch_counter_KiB: {out['FETCH_SIZE'][2]:.6e}  (copy calibration x{out['FETCH_SIZE'][1]:.4f})")
    print(f"write_counter_KiB: {out['WRITE_SIZE'][2]:.6e}  (copy calibration x{out['WRITE_SIZE'][1]:.4f})")


def sq(d, ring_slices):
    rs = float(ring_slices)
    tot, disp = {}, set()
    for r in _rows(os.path.join(d, "**", "*counter_collection.csv")):
        if "wake_march_kernel" not in r["Kernel_Name"]:
            continue
        tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.add((r["Counter_Name"], r["Dispatch_Id"]))
    print(f"source_digest: {source_digest()}")
    print(f"ring_slices: {rs:.6e}")
    print("| counter | sum | per ring-slice |")
    print("|---|---|---|")
    for k in sorted(tot):
        print(f"| {k} | {tot[k]:.4e} | {tot[k] / rs:.3f} |")
    w = tot.get("SQ_WAVE_CYCLES")
    if w:
        print()
        for k in ("SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_SCA",
                  "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS"):
            if k in tot:
                print(f"{k} / SQ_WAVE_CYCLES: {tot[k] / w:.3f}")
    if "SQ_INSTS_VALU" in tot:
        print(f"VALU lane-instructions per ring-slice (64 lanes): {tot['SQ_INSTS_VALU'] * 64 / rs:.0f}")
    if "SQ_INSTS_LDS" in tot:
        print(f"LDS instructions per ring-slice: {tot['SQ_INSTS_LDS'] / rs:.3f}")


def read_traffic(path, kernel="wake_march_kernel"):
    """Traffic figures of a summary file, if it belongs to the current sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if kv.get("source_digest") != source_digest(kernel):
        return None
    return kv


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4],
              kernel=sys.argv[5] if len(sys.argv) > 5 else "wake_march_kernel")
    elif sys.argv[1] == "stats":       # kernels by total time only (many dispatches)
        trace(sys.argv[2], sys.argv[3], sys.argv[4], per_dispatch=False)
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5],
                sys.argv[6] if len(sys.argv) > 6 else "wake_march_kernel")
    elif sys.argv[1] == "sq":
        sq(sys.argv[2], sys.argv[3])
