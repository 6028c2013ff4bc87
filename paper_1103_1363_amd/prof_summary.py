"""Summarise a rocprofv3 kernel trace (SQLite .db or kernel_trace.csv), or
turn two counter runs (FETCH_SIZE, WRITE_SIZE) into HBM bytes per launch.

Usage: python -m paper_1103_1363_amd.prof_summary TRACE [--top N] [--match REGEX]
       python -m paper_1103_1363_amd.prof_summary --pmc FETCH_CSV WRITE_CSV [--kernel SUBSTR]
       python -m paper_1103_1363_amd.prof_summary --counters CSV [CSV ...] [--match REGEX]

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


def summary(path, top=20, match=None):
    durs = load(path)
    rows = []
    for name, ds in durs.items():
        if match and not re.search(match, short(name)):
            continue
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


# Sources that define the single-lattice CG iteration kernels (cg_k1 ... cg_k5):
# their device code, the precision traits and loads they use, and the
# reduction helpers; with the compile flags, they fix the kernels' code.
KERNEL_SOURCES = ("solver_kernels.h", "dslash_core.h", "reduce.h", "lq_internal.h",
                  "site_index.h", "field_index.h")


def source_digest():
    """sha256 of the CG iteration kernels' sources and the compile flags
    (any change invalidates counter figures taken on an older build)."""
    import hashlib
    from paper_1103_1363_amd import build
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    h.update(" ".join(f for f in build.FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def pmc_counters(path, counter):
    """Per-dispatch totals of one counter: {kernel short name: [KiB per dispatch]}."""
    per = defaultdict(float)
    names = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            d = int(row["Dispatch_Id"])
            per[d] += float(row["Counter_Value"])
            names[d] = short(row["Kernel_Name"])
    out = defaultdict(list)
    for d, v in per.items():
        out[names[d]].append(v)
    return out


COPY_KERNELS = ("stream_copy_kernel", "__amd_rocclr_copyBuffer")
COPY_BYTES = 1 << 30  # the benchmark's reference copy: 1 GiB read and 1 GiB written


def copy_kernel(counts):
    """Name of the reference copy among the profiled kernels: the library's
    16-byte-per-lane streaming copy, else the runtime's copyBuffer."""
    for want in COPY_KERNELS:
        for name in counts:
            if want in name:
                return name
    raise KeyError("no reference copy kernel in the counter file")


def pmc_traffic(fetch_csv, write_csv, kernel=None):
    """HBM bytes per launch per kernel from FETCH_SIZE and WRITE_SIZE (KiB),
    each scaled so that the reference copy of COPY_BYTES reads and writes
    exactly that many bytes (the median dispatch of the copy kernel is taken
    as it)."""
    fetch = pmc_counters(fetch_csv, "FETCH_SIZE")
    write = pmc_counters(write_csv, "WRITE_SIZE")
    cf = COPY_BYTES / (statistics.median(fetch[copy_kernel(fetch)]) * 1024.0)
    cw = COPY_BYTES / (statistics.median(write[copy_kernel(write)]) * 1024.0)
    rows = []
    for name in sorted(fetch):
        if kernel and kernel not in name:
            continue
        f = statistics.median(fetch[name]) * 1024.0 * cf
        w = statistics.median(write.get(name, [0.0])) * 1024.0 * cw
        rows.append((name, len(fetch[name]), f, w))
    return cf, cw, rows


def counter_table(paths, match=None):
    """Median per dispatch of every counter in the counter files, per kernel:
    [(kernel, counter, dispatches, median)]."""
    rows = []
    for path in paths:
        with open(path) as f:
            counters = sorted({r["Counter_Name"] for r in csv.DictReader(f)})
        for c in counters:
            for name, vals in sorted(pmc_counters(path, c).items()):
                if match and not re.search(match, name):
                    continue
                rows.append((name, c, len(vals), statistics.median(vals)))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace", nargs="?")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--kernel")
    ap.add_argument("--match", help="regular expression on the short kernel name")
    ap.add_argument("--counters", nargs="+", metavar="CSV",
                    help="counter_collection.csv files: median of each counter per dispatch")
    a = ap.parse_args()
    if a.counters:
        print(f"# source_digest: {source_digest()}")
        print(f"{'kernel':40s} {'counter':36s} {'dispatches':>10s} {'per_dispatch':>14s}")
        for name, c, n, v in counter_table(a.counters, a.match):
            print(f"{name[:40]:40s} {c:36s} {n:10d} {v:14.6g}")
        return
    if a.pmc:
        cf, cw, rows = pmc_traffic(a.pmc[0], a.pmc[1], a.kernel)
        print(f"# counter scale (bytes per KiB counted): FETCH {cf:.3f}, WRITE {cw:.3f} "
              f"(from the {COPY_BYTES >> 20} MiB reference copy)")
        print(f"# source_digest: {source_digest()}")
        print(f"{'kernel':58s} {'dispatches':>10s} {'fetch_bytes':>14s} {'write_bytes':>14s}")
        for name, n, f, w in rows:
            print(f"{name[:58]:58s} {n:10d} {f:14.4g} {w:14.4g}")
        return
    print(f"# source: {os.path.basename(a.trace)} (durations in ns in the trace)")
    print(summary(a.trace, a.top, a.match))


if __name__ == "__main__":
    main()
