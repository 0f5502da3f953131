"""Markdown summaries of rocprofv3 output for the library's kernels.

  python -m paper_1801_08361_amd.rocprof_summary stats DIR
      per-kernel calls and durations from DIR's *kernel_stats.csv
      (rocprofv3 --kernel-trace --stats --output-format csv -d DIR)
  python -m paper_1801_08361_amd.rocprof_summary counters FETCH_DIR WRITE_DIR
      per-kernel FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the
      kernel's dispatches) from the *counter_collection.csv of two passes
      (rocprofv3 --pmc FETCH_SIZE ..., then --pmc WRITE_SIZE ...), each scaled
      by the factor that maps the counter's reading for the calibration
      kernel (the elementwise multiply among the run's first dispatches: one
      pass over 2^26 floats that reads 262144 KiB and writes 262144 KiB) to
      those known sizes
  python -m paper_1801_08361_amd.rocprof_summary valu PMC_DIR STATS_DIR
      per-kernel VALU instructions, lane utilisation, VALU busy and FP32 rate
      (rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU
      SQ_WAVES SQ_INSTS_VALU_FLOPS_FP32 ..., durations from a kernel trace of
      the same command)
  python -m paper_1801_08361_amd.rocprof_summary mfma PMC_DIR STATS_DIR
      per-kernel BF16 matrix FLOPs, rate and matrix-core busy
      (rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_BF16 ...)

Library kernels are those in namespace rl; parameter lists are dropped from
the names (template arguments are kept: k_b_score<4> and k_b_score<1> are
different kernels).
"""
from __future__ import annotations

import csv
import glob
import os
import sys
from collections import defaultdict

CAL_KIB = 262144.0


def _one(d: str, pattern: str) -> str:
    found = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not found:
        raise SystemExit(f"no {pattern} under {d}")
    return found[0]


def _short(name: str) -> str:
    name = name.replace("void ", "")
    name = name.split("(")[0]
    return name.replace("rl::", "")


def _is_lib(name: str) -> bool:
    return "rl::" in name


def stats(d: str) -> str:
    rows = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    out = ["| kernel | calls | total ms | avg us | min us | max us |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        if not _is_lib(r["Name"]):
            continue
        out.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} |")
    return "\n".join(out)


def _per_kernel(d: str):
    rows = list(csv.DictReader(open(_one(d, "*counter_collection.csv"))))
    key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else None
    if key:
        rows.sort(key=lambda r: int(r[key]))
    # the calibration kernel: the elementwise multiply among the run's first
    # dispatches (bench.py --copy-calibration runs it before anything else)
    cal = next((r for r in rows[:10] if not _is_lib(r["Kernel_Name"]) and "mul" in r["Kernel_Name"].lower()),
               None)
    if cal is None:
        raise SystemExit(f"no calibration kernel among the first dispatches in {d}")
    cal_kib = float(cal["Counter_Value"])
    factor = CAL_KIB / cal_kib
    lib = defaultdict(list)
    for r in rows:
        if _is_lib(r["Kernel_Name"]):
            lib[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in lib.items()}, cal_kib, factor


def counters(fetch_dir: str, write_dir: str) -> str:
    f, f_cal, f_fac = _per_kernel(fetch_dir)
    w, w_cal, w_fac = _per_kernel(write_dir)
    out = ["| counter | calibration kernel reads (KiB) | known (KiB) | factor |", "|---|---:|---:|---:|",
           f"| FETCH_SIZE | {f_cal:.1f} | {CAL_KIB:.0f} | {f_fac:.5f} |",
           f"| WRITE_SIZE | {w_cal:.1f} | {CAL_KIB:.0f} | {w_fac:.5f} |", "",
           "| kernel | dispatches | fetch KiB | write KiB | total MB |", "|---|---:|---:|---:|---:|"]
    for k in sorted(set(f) | set(w)):
        fk = f.get(k, (0.0, 0))[0] * f_fac
        wk = w.get(k, (0.0, 0))[0] * w_fac
        n = max(f.get(k, (0, 0))[1], w.get(k, (0, 0))[1])
        out.append(f"| {k} | {n} | {fk:.0f} | {wk:.0f} | {(fk + wk) * 1024 / 1e6:.2f} |")
    return "\n".join(out)


def valu(pmc_dir: str, stats_dir: str) -> str:
    """VALU use per kernel: mean per dispatch of SQ_INSTS_VALU and SQ_WAVES;
    lane utilisation SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU); VALU
    busy 4 SQ_INSTS_VALU / (1024 SIMDs x 2.4 GHz x the kernel's average
    duration in the kernel trace of stats_dir); FP32 rate 64
    SQ_INSTS_VALU_FLOPS_FP32 / that duration."""
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(_one(pmc_dir, "*counter_collection.csv"))):
        if _is_lib(r["Kernel_Name"]):
            vals[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = {}
    for r in csv.DictReader(open(_one(stats_dir, "*kernel_stats.csv"))):
        if _is_lib(r["Name"]):
            k = _short(r["Name"])
            n0, t0 = dur.get(k, (0, 0.0))
            dur[k] = (n0 + int(r["Calls"]), t0 + float(r["TotalDurationNs"]))
    out = ["| kernel | dispatches | VALU instr. | waves | per wave | lane utilisation | VALU busy | FP32 TFLOP/s |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    mean = lambda v: sum(v) / len(v) if v else 0.0
    for k in sorted(vals, key=lambda k: -mean(vals[k]["SQ_INSTS_VALU"])):
        c = vals[k]
        iv, wv = mean(c["SQ_INSTS_VALU"]), mean(c["SQ_WAVES"])
        act, thr = mean(c["SQ_ACTIVE_INST_VALU"]), mean(c["SQ_THREAD_CYCLES_VALU"])
        n, tot = dur.get(k, (0, 0.0))
        avg_s = tot / n * 1e-9 if n else 0.0
        busy = 4 * iv / (1024 * 2.4e9 * avg_s) if avg_s else 0.0
        fl = 64 * mean(c["SQ_INSTS_VALU_FLOPS_FP32"]) / avg_s / 1e12 if avg_s else 0.0
        util = thr / (64 * act) if act else 0.0
        out.append(f"| {k} | {len(c['SQ_INSTS_VALU'])} | {iv:,.0f} | {wv:,.0f} | {iv / wv if wv else 0:,.0f} | "
                   f"{100 * util:.1f} % | {100 * busy:.1f} % | {fl:.2f} |")
    return "\n".join(out)


def mfma(pmc_dir: str, stats_dir: str) -> str:
    """Matrix-core use per kernel: BF16 FLOPs = 512 SQ_INSTS_VALU_MFMA_MOPS_BF16
    per dispatch (mean; the counter's unit is 512 FLOPs), the rate over the
    kernel's average duration in the kernel trace of stats_dir, and
    matrix-core busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x 2.4 GHz x
    that duration)."""
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(_one(pmc_dir, "*counter_collection.csv"))):
        if _is_lib(r["Kernel_Name"]):
            vals[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = {}
    for r in csv.DictReader(open(_one(stats_dir, "*kernel_stats.csv"))):
        if _is_lib(r["Name"]):
            k = _short(r["Name"])
            n0, t0 = dur.get(k, (0, 0.0))
            dur[k] = (n0 + int(r["Calls"]), t0 + float(r["TotalDurationNs"]))
    out = ["| kernel | dispatches | MFLOP per dispatch | avg us | TFLOP/s | of 2.5 PFLOP/s | matrix-core busy |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    mean = lambda v: sum(v) / len(v) if v else 0.0
    for k in sorted(vals):
        c = vals[k]
        fl = 512 * mean(c["SQ_INSTS_VALU_MFMA_MOPS_BF16"])
        if fl == 0:
            continue
        n, tot = dur.get(k, (0, 0.0))
        avg_s = tot / n * 1e-9 if n else 0.0
        rate = fl / avg_s / 1e12 if avg_s else 0.0
        busy = mean(c["SQ_VALU_MFMA_BUSY_CYCLES"]) / (1024 * 2.4e9 * avg_s) if avg_s else 0.0
        out.append(f"| {k} | {len(c['SQ_INSTS_VALU_MFMA_MOPS_BF16'])} | {fl / 1e6:.1f} | {avg_s * 1e6:.2f} | "
                   f"{rate:.2f} | {100 * rate / 2500:.2f} % | {100 * busy:.2f} % |")
    return "\n".join(out)


def main(argv) -> None:
    if len(argv) == 2 and argv[0] == "stats":
        print(stats(argv[1]))
    elif len(argv) == 3 and argv[0] == "counters":
        print(counters(argv[1], argv[2]))
    elif len(argv) == 3 and argv[0] == "valu":
        print(valu(argv[1], argv[2]))
    elif len(argv) == 3 and argv[0] == "mfma":
        print(mfma(argv[1], argv[2]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
