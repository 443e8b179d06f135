"""Summarise rocprofv3 CSV output into a short text table.

  python -m paper_1210_0748_amd.profsum stats   <kernel_stats.csv> [--top N]
  python -m paper_1210_0748_amd.profsum rounds  <kernel_trace.csv>
  python -m paper_1210_0748_amd.profsum counters <counter_collection.csv> --kernel SUBSTR
  python -m paper_1210_0748_amd.profsum traffic <fetch.csv> --write W.csv --cal-fetch CF.csv
         --cal-write CW.csv --kernel SUBSTR --name NAME --out profiles/traffic.json
         (NAME: the kernel class, or CLASS@WORKLOAD beside the entry of another workload)
         [--workload W --k-cap K --no-early-stop]   (the bench job the counters ran)
  python -m paper_1210_0748_amd.profsum gbs <kernel_stats.csv> --fetch F.csv --write W.csv
         [--scales profiles/traffic.json] [--top N]

`traffic` turns FETCH_SIZE / WRITE_SIZE runs of a command and of the 1 GiB
copy probe (`bench.py --copy-probe`) into bytes per launch of one
kernel, stamped with a digest of the kernel sources (bench.py reports the
figure only while the digest matches). `stats` lists kernels by total time; `rounds` splits a kernel trace into
refinement rounds (at each launch of the signature kernel) and
reports busy time, span and launch counts; `counters` averages the PMC
values (e.g. FETCH_SIZE, WRITE_SIZE in KiB) per dispatch of the kernels whose
name contains SUBSTR. `gbs` joins a kernel-statistics run with FETCH_SIZE and
WRITE_SIZE runs of the same command: per kernel the measured HBM bytes per
dispatch (scaled by the copy-probe factors of `--scales`) over its average
duration, and that rate as a fraction of the 8 TB/s peak.
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
    marks = [i for i, r in enumerate(rows) if "signature_k" in r["Kernel_Name"]]
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


def _per_kernel_mean(path):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def cmd_gbs(stats_path, fetch_path, write_path, scales_path, top, peak_gbs=8000.0):
    import json
    with open(scales_path) as fh:
        t = json.load(fh)
    fs, ws = float(t["fetch_scale"]), float(t["write_scale"])
    fetch, write = _per_kernel_mean(fetch_path), _per_kernel_mean(write_path)
    rows = list(csv.DictReader(open(stats_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("%-60s %6s %9s %10s %10s %8s %6s" % ("kernel", "calls", "avg_us", "fetch_MB", "write_MB", "GB/s",
                                                "of_8TB"))
    for r in rows[:top] if top > 0 else rows:
        name = r["Name"]
        if name not in fetch or name not in write:
            continue
        fb = fetch[name] * 1024.0 * fs
        wb = write[name] * 1024.0 * ws
        avg_ns = float(r["AverageNs"])
        gbs = (fb + wb) / avg_ns if avg_ns > 0 else 0.0
        print("%-60s %6s %9.1f %10.2f %10.2f %8.0f %6.3f" % (short(name, 60), r["Calls"], avg_ns / 1e3, fb / 1e6,
                                                             wb / 1e6, gbs, gbs / peak_gbs))


def _values(path, kernel):
    rows = list(csv.DictReader(open(path)))
    return [float(r["Counter_Value"]) for r in rows if kernel in r.get("Kernel_Name", "")]


def source_digest():
    import hashlib
    import os
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cmd_traffic(a):
    import json
    import os
    copy_bytes = float(1 << 30)
    # the copy probe moves 1 GiB each way; counters are in KiB
    cal_f = max(_values(a.cal_fetch, "copyBuffer") or _values(a.cal_fetch, ""))
    cal_w = max(_values(a.cal_write, "copyBuffer") or _values(a.cal_write, ""))
    fscale = copy_bytes / (cal_f * 1024.0)
    wscale = copy_bytes / (cal_w * 1024.0)
    f = _values(a.csv, a.kernel)
    w = _values(a.write, a.kernel)
    fb = sum(f) * 1024.0 * fscale / len(f)
    wb = sum(w) * 1024.0 * wscale / len(w)
    t = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            t = json.load(fh)
    if t.get("source_digest") != source_digest():
        t = {"kernels": {}}
    t["source_digest"] = source_digest()
    t["fetch_scale"] = fscale
    t["write_scale"] = wscale
    t["note"] = ("rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch), averaged over the dispatches of "
                 "the kernel, scaled by the readings of a 1 GiB device copy")
    t.setdefault("kernels", {})[a.name] = {
        "kernel": a.kernel, "launches": len(f),
        # the bench job the counters were read on
        "workload": a.workload, "early_stop": not a.no_early_stop, "k_cap": a.k_cap,
        "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb,
        "fetch_bytes_per_dispatch": [x * 1024.0 * fscale for x in f],
        "write_bytes_per_dispatch": [x * 1024.0 * wscale for x in w]}
    with open(a.out, "w") as fh:
        json.dump(t, fh, indent=1)
    print("%s: %.3g B fetched + %.3g B written per launch (%d launches)" % (a.name, fb, wb, len(f)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "rounds", "counters", "traffic", "gbs"])
    ap.add_argument("csv")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--kernel", default="")
    ap.add_argument("--write", default=None)
    ap.add_argument("--fetch", default=None)
    ap.add_argument("--scales", default="profiles/traffic.json")
    ap.add_argument("--cal-fetch", default=None)
    ap.add_argument("--cal-write", default=None)
    ap.add_argument("--name", default=None)
    ap.add_argument("--out", default="profiles/traffic.json")
    ap.add_argument("--workload", default="powerlaw-10M-100M", help="traffic: the bench job's workload")
    ap.add_argument("--k-cap", type=int, default=10, help="traffic: the bench job's k")
    ap.add_argument("--no-early-stop", action="store_true", help="traffic: the bench job ran without early stop")
    a = ap.parse_args(argv)
    if a.mode == "stats":
        cmd_stats(a.csv, a.top)
    elif a.mode == "rounds":
        cmd_rounds(a.csv)
    elif a.mode == "counters":
        cmd_counters(a.csv, a.kernel)
    elif a.mode == "gbs":
        cmd_gbs(a.csv, a.fetch, a.write, a.scales, a.top if a.top != 25 else 0)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    sys.exit(main())
