"""Summarise a rocprofv3 kernel trace (SQLite .db or kernel_trace.csv).

Usage: python -m paper_1103_1363_amd.prof_summary TRACE [--top N]

For every kernel: launches, total and average duration, and the average over
"working" launches only.  The solvers replay captured graphs of several CG
iterations; replays past the point where the solve stopped launch kernels
that return at once (a few microseconds), which pull the plain average
down.  A launch counts as working when it lasts at least a quarter of that
kernel's median duration.
"""
from __future__ import annotations

import argparse
import csv
import os
import re
import sqlite3
import statistics
from collections import defaultdict


def load(path):
    durs = defaultdict(list)
    if path.endswith(".db"):
        c = sqlite3.connect(path)
        for name, d in c.execute("select name, duration from kernels"):
            durs[name].append(float(d))
    else:
        with open(path) as f:
            for row in csv.DictReader(f):
                d = float(row["End_Timestamp"]) - float(row["Start_Timestamp"])
                durs[row["Kernel_Name"]].append(d)
    return durs


def short(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("lq::", "")
    return re.sub(r"\(.*", "", name)


def summary(path, top=20):
    durs = load(path)
    rows = []
    for name, ds in durs.items():
        med = statistics.median(ds)
        work = [d for d in ds if d >= 0.25 * med]
        rows.append((sum(ds), short(name), len(ds), sum(ds) / len(ds), len(work),
                     sum(work) / len(work)))
    rows.sort(reverse=True)
    total = sum(r[0] for r in rows)
    out = [f"{'kernel':58s} {'calls':>6s} {'total_ms':>9s} {'avg_us':>9s} "
           f"{'work_calls':>10s} {'work_avg_us':>11s} {'share':>6s}"]
    for tot, name, n, avg, nw, wavg in rows[:top]:
        out.append(f"{name[:58]:58s} {n:6d} {tot / 1e6:9.2f} {avg / 1e3:9.2f} {nw:10d} "
                   f"{wavg / 1e3:11.2f} {100 * tot / total:5.1f}%")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--top", type=int, default=20)
    a = ap.parse_args()
    print(f"# source: {os.path.basename(a.trace)} (durations in ns in the trace)")
    print(summary(a.trace, a.top))


if __name__ == "__main__":
    main()
