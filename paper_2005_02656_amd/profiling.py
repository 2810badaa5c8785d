"""Summaries of rocprofv3 output for the kernels of one workload.

    python -m paper_2005_02656_amd.profiling --trace DIR [--fetch DIR --write DIR
        --calib-bytes N] [--l2 DIR] [--sq DIR] [--mem DIR] --kernel k_candidates
        --workload c4 --command "..." --out FILE

Reads the CSV output of `rocprofv3 --kernel-trace --stats` (per-kernel call
counts and durations) and, optionally, of `rocprofv3 --pmc` runs of the same
command: FETCH_SIZE and WRITE_SIZE (HBM bytes), TCC_HIT_sum and TCC_MISS_sum
(L2 hit rate), and SQ_INSTS_VALU, SQ_INSTS_VALU_FLOPS_FP64,
SQ_INSTS_VALU_FLOPS_FP32, SQ_WAVES, VALUBusy and OccupancyPercent (vector
instructions, counted flops, VALU busy and occupancy), and the L1/address
path: TA_BUSY_avr, TA_ADDR_STALLED_BY_TC_CYCLES_sum, TCP_TOTAL_CACHE_ACCESSES_sum,
TCP_TCC_READ_REQ_sum, TCP_TCC_READ_REQ_LATENCY_sum and GRBM_GUI_ACTIVE (how busy
the texture addresser is, the L1 hit rate and the L2 latency the L1 sees).
The byte counters are scaled by what they read for a device copy of known size
in the same run (the runtime's copy kernel), per counter, and reported per
launch.  The summary
records a digest of the library sources so that a reader (bench.py) can tell
whether the counters still describe the kernels that are built.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CALIB_KERNEL = "__amd_rocclr_copyBuffer"


def source_digest() -> str:
    """sha256 over the HIP sources and the public header (sorted by name)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*")) +
                   [os.path.join(ROOT, "include", "sph.h")])
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    m = re.search(r"(k_\w+)(?:<[^>]*>)?\(", name)
    if m:
        return m.group(1)
    m = re.search(r"(__amd_rocclr_\w+)", name)
    return m.group(1) if m else name.split("(")[0][:60]


def _one(pattern):
    got = glob.glob(pattern, recursive=True)
    if not got:
        raise FileNotFoundError(pattern)
    return got[0]


# the L1/address-path pass: 2 TA, 4 TCP and 1 GRBM counters fit one run.
# GRBM_GUI_ACTIVE comes summed over the chip's 8 XCDs (8 times the kernel's
# clock cycles); TA_BUSY_avr is per TA (one per CU) and the _sum counters add
# the 256 CUs' values.
XCDS, CUS = 8, 256
MEM_COUNTERS = ("TA_BUSY_avr", "TA_ADDR_STALLED_BY_TC_CYCLES_sum", "TCP_TOTAL_CACHE_ACCESSES_sum",
                "TCP_TCC_READ_REQ_sum", "TCP_TCC_READ_REQ_LATENCY_sum", "GRBM_GUI_ACTIVE")


def kernel_stats(trace_dir: str) -> list:
    """[(kernel, calls, mean_ms, total_ms, percent)] from the kernel_stats CSV."""
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))))
    out = []
    for r in rows:
        out.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e6,
                    float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    out.sort(key=lambda t: -t[3])
    return out


def counter_means(pmc_dir: str, counter: str) -> dict:
    """{kernel: [values per dispatch]} of one counter (KiB as rocprofv3 reports)."""
    f = _one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    vals = {}
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def calibrated_bytes(pmc_dir: str, counter: str, calib_bytes: int):
    """Per-kernel mean bytes per dispatch and the scale factor: the copy of
    calib_bytes read and wrote exactly that many bytes, so the counter's reading
    for it (the largest copy dispatch) fixes the factor."""
    vals = counter_means(pmc_dir, counter)
    calib = max(vals.get(CALIB_KERNEL, [0.0]))
    if calib <= 0:
        raise RuntimeError(f"no {CALIB_KERNEL} dispatch in {pmc_dir}")
    factor = calib_bytes / (calib * 1024.0)
    return {k: statistics.fmean(v) * 1024.0 * factor for k, v in vals.items()}, factor


def summary(args) -> str:
    st = kernel_stats(args.trace)
    lines = [f"# {args.kernel} — {args.workload}", "",
             f"command: `{args.command}`", f"source_digest: {source_digest()}", "",
             "## Kernel trace (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | mean ms | total ms | % |", "|---|---|---|---|---|"]
    for k, c, m, t, p in st[:args.top]:
        lines.append(f"| {k} | {c} | {m:.3f} | {t:.1f} | {p:.2f} |")
    dom = [t for t in st if t[0] == args.kernel]
    if dom:
        lines += ["", f"mean_ms_per_launch: {dom[0][2]:.4f}"]
    if args.fetch and args.write:
        fb, ff = calibrated_bytes(args.fetch, "FETCH_SIZE", args.calib_bytes)
        wb, wf = calibrated_bytes(args.write, "WRITE_SIZE", args.calib_bytes)
        lines += ["", "## HBM bytes per launch (rocprofv3 --pmc, calibrated)", "",
                  f"calibration: a {args.calib_bytes} B device copy ({CALIB_KERNEL}); "
                  f"FETCH_SIZE factor {ff:.4f}, WRITE_SIZE factor {wf:.4f}", "",
                  "| kernel | fetch GB | write GB |", "|---|---|---|"]
        names = sorted(set(fb) | set(wb), key=lambda k: -(fb.get(k, 0) + wb.get(k, 0)))
        for k in names[:args.top]:
            lines.append(f"| {k} | {fb.get(k, 0) / 1e9:.3f} | {wb.get(k, 0) / 1e9:.3f} |")
        if args.kernel in fb:
            lines += ["", f"fetch_bytes_per_launch: {fb[args.kernel]:.6e}",
                      f"write_bytes_per_launch: {wb.get(args.kernel, 0.0):.6e}"]
    kern_rows = [t[0] for t in st if t[0].startswith("k_")][:args.top]
    if args.l2:
        hit, miss = counter_means(args.l2, "TCC_HIT_sum"), counter_means(args.l2, "TCC_MISS_sum")
        lines += ["", "## L2 (rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum)", "",
                  "| kernel | hit rate | requests per launch |", "|---|---|---|"]
        for k in kern_rows:
            if k in hit and k in miss:
                h, mi = statistics.fmean(hit[k]), statistics.fmean(miss[k])
                lines.append(f"| {k} | {h / max(h + mi, 1):.3f} | {h + mi:.4e} |")
        if args.kernel in hit and args.kernel in miss:
            h, mi = statistics.fmean(hit[args.kernel]), statistics.fmean(miss[args.kernel])
            lines += ["", f"l2_hit_rate: {h / max(h + mi, 1):.4f}"]
    if args.sq:
        cs = {c: counter_means(args.sq, c) for c in
              ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP32",
               "SQ_WAVES", "VALUBusy", "OccupancyPercent")}
        lines += ["", "## Vector ALU (rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_VALU_FLOPS_FP64 "
                  "SQ_INSTS_VALU_FLOPS_FP32 SQ_WAVES VALUBusy OccupancyPercent)", "",
                  "| kernel | VALU insts per wave | FP64 flops per launch | FP32 flops per launch "
                  "| VALU busy % | occupancy % |", "|---|---|---|---|---|---|"]
        mean = lambda c, k: statistics.fmean(cs[c][k]) if k in cs[c] else float("nan")
        for k in kern_rows:
            if k not in cs["SQ_INSTS_VALU"]:
                continue
            w = mean("SQ_WAVES", k)
            lines.append(f"| {k} | {mean('SQ_INSTS_VALU', k) / max(w, 1):.0f} | "
                         f"{mean('SQ_INSTS_VALU_FLOPS_FP64', k):.4e} | "
                         f"{mean('SQ_INSTS_VALU_FLOPS_FP32', k):.4e} | "
                         f"{mean('VALUBusy', k):.1f} | {mean('OccupancyPercent', k):.1f} |")
        k = args.kernel
        if k in cs["SQ_INSTS_VALU"]:
            # the FLOPS counters count each wavefront instruction once: times
            # the 64 lanes they are lane flops (k_integrate: 56 per particle,
            # its arithmetic counted by hand)
            lines += ["", f"valu_insts_per_wave: {mean('SQ_INSTS_VALU', k) / max(mean('SQ_WAVES', k), 1):.1f}",
                      f"fp64_flops_per_launch: {mean('SQ_INSTS_VALU_FLOPS_FP64', k):.6e}",
                      f"fp64_lane_flops_per_launch: {64 * mean('SQ_INSTS_VALU_FLOPS_FP64', k):.6e}",
                      f"valu_busy_percent: {mean('VALUBusy', k):.2f}",
                      f"occupancy_percent: {mean('OccupancyPercent', k):.2f}"]
    if args.mem:
        cs = {c: counter_means(args.mem, c) for c in MEM_COUNTERS}
        lines += ["", "## L1 and address path (rocprofv3 --pmc " + " ".join(MEM_COUNTERS) + ")",
                  "", "| kernel | TA busy % | TA stalled by L1 % | L1 hit rate | "
                  "L1 accesses per launch | L1 to L2 reads per launch | L2 read latency (cycles) |",
                  "|---|---|---|---|---|---|---|"]
        mean = lambda c, k: statistics.fmean(cs[c][k]) if k in cs[c] else float("nan")
        for k in kern_rows:
            if k not in cs["GRBM_GUI_ACTIVE"]:
                continue
            cyc = max(mean("GRBM_GUI_ACTIVE", k) / XCDS, 1.0)
            acc, req = mean("TCP_TOTAL_CACHE_ACCESSES_sum", k), mean("TCP_TCC_READ_REQ_sum", k)
            lines.append(f"| {k} | {100 * mean('TA_BUSY_avr', k) / cyc:.1f} | "
                         f"{100 * mean('TA_ADDR_STALLED_BY_TC_CYCLES_sum', k) / (CUS * cyc):.1f} | "
                         f"{1 - req / max(acc, 1):.3f} | {acc:.4e} | {req:.4e} | "
                         f"{mean('TCP_TCC_READ_REQ_LATENCY_sum', k) / max(req, 1):.0f} |")
        k = args.kernel
        if k in cs["GRBM_GUI_ACTIVE"]:
            cyc = max(mean("GRBM_GUI_ACTIVE", k) / XCDS, 1.0)
            acc, req = mean("TCP_TOTAL_CACHE_ACCESSES_sum", k), mean("TCP_TCC_READ_REQ_sum", k)
            lines += ["", f"ta_busy_percent: {100 * mean('TA_BUSY_avr', k) / cyc:.2f}",
                      f"ta_stalled_by_l1_percent: "
                      f"{100 * mean('TA_ADDR_STALLED_BY_TC_CYCLES_sum', k) / (CUS * cyc):.2f}",
                      f"l1_accesses_per_launch: {acc:.6e}",
                      f"l1_hit_rate: {1 - req / max(acc, 1):.4f}",
                      f"l2_read_latency_cycles: {mean('TCP_TCC_READ_REQ_LATENCY_sum', k) / max(req, 1):.1f}"]
    return "\n".join(lines) + "\n"


def read_summary(path: str) -> dict:
    """key: value lines of a summary written by this module."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        m = re.match(r"^(\w+): (\S+)\s*$", line.strip())
        if m:
            out[m.group(1)] = m.group(2)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-bytes", type=int, default=0)
    ap.add_argument("--l2", help="rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum output")
    ap.add_argument("--sq", help="rocprofv3 --pmc SQ_INSTS_VALU ... OccupancyPercent output")
    ap.add_argument("--mem", help="rocprofv3 --pmc " + " ".join(MEM_COUNTERS) + " output")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--top", type=int, default=16)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    text = summary(args)
    with open(args.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
