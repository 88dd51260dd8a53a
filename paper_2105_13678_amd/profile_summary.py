"""Short text summaries of rocprofv3 output for libpa's kernels.

    python -m paper_2105_13678_amd.profile_summary stats TRACE_DIR
        per-kernel call count, average and median duration from a
        `rocprofv3 --kernel-trace --stats --output-format csv -o run` directory

    python -m paper_2105_13678_amd.profile_summary hbm FETCH_DIR WRITE_DIR --calib-bytes BYTES
        HBM bytes per launch from two `rocprofv3 --pmc FETCH_SIZE` /
        `--pmc WRITE_SIZE` directories of the same program.  The program ends
        with a plain device copy of BYTES/2 bytes (bench.py --calib-copy-mib);
        the ratio of its true read (write) bytes to what FETCH_SIZE
        (WRITE_SIZE) reports for it scales every other kernel's counter.

    python -m paper_2105_13678_amd.profile_summary valu SQ_DIR
        per-kernel VALU instruction counts and issue utilisation from a
        `rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU
        SQ_BUSY_CYCLES ...` directory (per kernel the counts of its largest
        launch and the median duration of the launches with those counts)

Kernel names are shortened (namespaces and argument lists dropped, template
arguments kept).  Output is Markdown on stdout.
"""
from __future__ import annotations

import argparse
import collections
import csv
import os
import re

from .build import source_digest


def short_name(name: str) -> str:
    m = re.search(r"at::native::\w*elementwise_kernel<.*FillFunctor<(\w+)>", name)
    if m:  # torch's fill of the benchmark's output and status buffers
        return {"long": "torch fill (int64)", "int": "torch fill (int32)"}.get(m.group(1), "torch fill")
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"^void ", "", name)
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _durations(trace_dir: str):
    """Per-kernel launch durations (ns) from run_kernel_trace.csv, if present."""
    path = os.path.join(trace_dir, "run_kernel_trace.csv")
    out = collections.defaultdict(list)
    if os.path.exists(path):
        for r in csv.DictReader(open(path)):
            out[short_name(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def _median(v):
    v = sorted(v)
    n = len(v)
    return (v[n // 2] + v[(n - 1) // 2]) / 2 if n else float("nan")


def stats(trace_dir: str) -> str:
    rows = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    durs = _durations(trace_dir)
    lines = ["| kernel | calls | average µs | median µs | min µs | max µs | share of GPU time |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        nm = short_name(r["Name"])
        lines.append(f"| `{nm}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{_median(durs.get(nm, [])) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}% |")
    return "\n".join(lines)


def _per_dispatch(pmc_dir: str):
    rows = list(csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))))
    agg = collections.OrderedDict()
    for r in rows:
        key = (int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]))
        agg[key] = agg.get(key, 0.0) + float(r["Counter_Value"])  # KiB, summed over XCDs/channels
    return agg


def hbm(fetch_dir: str, write_dir: str, calib_bytes: int) -> str:
    fe, wr = _per_dispatch(fetch_dir), _per_dispatch(write_dir)
    # the calibration copy is the program's last dispatch
    (fk, fcal), (wk, wcal) = list(fe.items())[-1], list(wr.items())[-1]
    f_scale = (calib_bytes / 2) / (fcal * 1024)
    w_scale = (calib_bytes / 2) / (wcal * 1024)
    by = collections.OrderedDict()
    for (d, nm), v in list(fe.items())[:-1]:
        by.setdefault(nm, [[], []])[0].append(v * 1024 * f_scale)
    for (d, nm), v in list(wr.items())[:-1]:
        by.setdefault(nm, [[], []])[1].append(v * 1024 * w_scale)
    lines = [f"Calibration: plain copy of {calib_bytes // 2} bytes ({fk[1]}): FETCH_SIZE read "
             f"{fcal:.1f} KiB, WRITE_SIZE read {wcal:.1f} KiB, so FETCH bytes = FETCH_SIZE KiB x 1024 x "
             f"{f_scale:.4f} and WRITE bytes = WRITE_SIZE KiB x 1024 x {w_scale:.4f}.",
             "",
             "| kernel | launches | HBM read MiB / launch | HBM write MiB / launch |",
             "|---|---:|---:|---:|"]
    for nm, (f, w) in by.items():
        if not f:
            continue
        lines.append(f"| `{nm}` | {len(f)} | {sum(f) / len(f) / 2**20:.2f} | "
                     f"{(sum(w) / len(w) / 2**20) if w else float('nan'):.2f} |")
    lines.append("")
    lines.append("Machine-readable (bytes per launch, averaged; `sources` = digest of the library sources "
                 "the counters were taken on):")
    lines.append("")
    digest = source_digest()
    for nm, (f, w) in by.items():
        if f and w:
            key = re.sub(r"[ ()]+", "_", nm).strip("_") if " " in nm else nm
            lines.append(f"    traffic {key} fetch={sum(f) / len(f):.0f} write={sum(w) / len(w):.0f} "
                         f"sources={digest}")
    return "\n".join(lines)


def valu(sq_dir: str, cus: int = 256, simds: int = 4, ghz: float = 2.4) -> str:
    """VALU issue utilisation = wave-level VALU instructions x 4 cycles (a
    64-lane instruction occupies a 16-lane SIMD for 4 cycles) / (duration x
    clock x SIMDs).  Durations are those of the counting run, which the
    profiler lengthens somewhat."""
    rows = list(csv.DictReader(open(os.path.join(sq_dir, "run_counter_collection.csv"))))
    agg, dur = collections.OrderedDict(), {}
    for r in rows:
        key = (int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]))
        c = agg.setdefault(key, collections.defaultdict(float))
        c[r["Counter_Name"]] += float(r["Counter_Value"])
        dur[key] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    # per kernel: the counts of its largest launch (most VALU instructions;
    # the launches of a hash kernel all have the same counts) and the median
    # duration of the launches with those counts
    top = {}
    for key, c in agg.items():
        if key[1] not in top or c["SQ_INSTS_VALU"] > agg[top[key[1]]]["SQ_INSTS_VALU"]:
            top[key[1]] = key
    med = collections.defaultdict(list)
    for key, ns in dur.items():
        if agg[key]["SQ_INSTS_VALU"] == agg[top[key[1]]]["SQ_INSTS_VALU"]:
            med[key[1]].append(ns)
    lines = ["| kernel | µs (counting run, median) | waves | VALU instr (wave) | VALU issue util | LDS instr | LDS bank conflicts |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    seen = set()
    for key0 in agg:
        if key0[1] in seen:
            continue
        seen.add(key0[1])
        key = top[key0[1]]
        c = agg[key]
        ns = _median(med[key[1]])
        util = c["SQ_INSTS_VALU"] * 4 / (ns * ghz * cus * simds) if ns else 0.0
        lines.append(f"| `{key[1]}` | {ns / 1e3:.1f} | {c['SQ_WAVES']:.0f} | {c['SQ_INSTS_VALU']:.4g} | {util:.2f} | "
                     f"{c['SQ_INSTS_LDS']:.4g} | {c['SQ_LDS_BANK_CONFLICT']:.4g} |")
    return "\n".join(lines)


def read_traffic(path: str, kernel: str):
    """(fetch_bytes, write_bytes) for `kernel` from a summary written by
    `hbm`, or None when absent or taken on other sources than the current
    ones."""
    if not os.path.exists(path):
        return None
    digest = source_digest()
    for line in open(path):
        m = re.match(r"\s*traffic (\S+) fetch=(\d+) write=(\d+) sources=([0-9a-f]+)", line)
        if m and m.group(1) == kernel and m.group(4) == digest:
            return int(m.group(2)), int(m.group(3))
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace_dir")
    h = sub.add_parser("hbm")
    h.add_argument("fetch_dir")
    h.add_argument("write_dir")
    h.add_argument("--calib-bytes", type=int, required=True)
    v = sub.add_parser("valu")
    v.add_argument("sq_dir")
    a = ap.parse_args()
    if a.cmd == "stats":
        print(stats(a.trace_dir))
    elif a.cmd == "hbm":
        print(hbm(a.fetch_dir, a.write_dir, a.calib_bytes))
    else:
        print(valu(a.sq_dir))


if __name__ == "__main__":
    main()
