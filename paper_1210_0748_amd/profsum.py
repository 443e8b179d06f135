"""Summarise rocprofv3 CSV output into a short text table.

  python -m paper_1210_0748_amd.profsum stats   <kernel_stats.csv> [--top N]
  python -m paper_1210_0748_amd.profsum rounds  <kernel_trace.csv>
  python -m paper_1210_0748_amd.profsum counters <counter_collection.csv> --kernel SUBSTR

`stats` lists kernels by total time; `rounds` splits a kernel trace into
refinement rounds (at each launch of the thread-bucket signature kernel) and
reports busy time, span and launch counts; `counters` averages the PMC
values (e.g. FETCH_SIZE, WRITE_SIZE in KiB) per dispatch of the kernels whose
name contains SUBSTR.
"""
from __future__ import annotations

import argparse
import csv
import re
import sys
from collections import defaultdict


def short(name, width=70):
    name = re.sub(r"\(.*", "", name)
    name = name.replace("void ", "").replace("kb::", "")
    return name[:width]


def cmd_stats(path, top):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print("%-70s %6s %10s %10s %10s %6s" % ("kernel", "calls", "total_ms", "avg_us", "max_us", "pct"))
    for r in rows[:top]:
        t = float(r["TotalDurationNs"])
        print("%-70s %6s %10.3f %10.1f %10.1f %6.2f" % (short(r["Name"]), r["Calls"], t / 1e6,
                                                      float(r["AverageNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                                                      100.0 * t / total))
    print("all kernels: %.3f ms" % (total / 1e6))


def cmd_rounds(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if "sig_thread_k" in r["Kernel_Name"] or "signature_k" in r["Kernel_Name"]]
    print("%5s %10s %10s %10s" % ("round", "launches", "busy_ms", "span_ms"))
    for j, (a, b) in enumerate(zip(marks, marks[1:] + [len(rows)])):
        seg = rows[a:b]
        busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in seg)
        span = int(seg[-1]["End_Timestamp"]) - int(seg[0]["Start_Timestamp"])
        print("%5d %10d %10.3f %10.3f" % (j, len(seg), busy / 1e6, span / 1e6))


def cmd_counters(path, kernel):
    rows = list(csv.DictReader(open(path)))
    acc = defaultdict(list)
    for r in rows:
        if kernel in r.get("Kernel_Name", ""):
            acc[r["Counter_Name"]].append(float(r["Counter_Value"]))
    for name, vals in sorted(acc.items()):
        print("%-14s dispatches %5d  mean %14.1f  max %14.1f" % (name, len(vals), sum(vals) / len(vals), max(vals)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "rounds", "counters"])
    ap.add_argument("csv")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--kernel", default="")
    a = ap.parse_args(argv)
    if a.mode == "stats":
        cmd_stats(a.csv, a.top)
    elif a.mode == "rounds":
        cmd_rounds(a.csv)
    else:
        cmd_counters(a.csv, a.kernel)


if __name__ == "__main__":
    sys.exit(main())
