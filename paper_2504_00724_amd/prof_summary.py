"""Summaries of rocprofv3 output as short Markdown tables.

    python3 -m paper_2504_00724_amd.prof_summary trace STATS.csv|RESULTS.db
    python3 -m paper_2504_00724_amd.prof_summary pmc FETCH.csv WRITE.csv \
        --cells N --kernel NAME [--calib-kernel k_copy]
    python3 -m paper_2504_00724_amd.prof_summary cycle KERNEL_TRACE.csv

``trace`` reads a ``--kernel-trace --stats`` run (the ``*_kernel_stats.csv``
of ``--output-format csv``, or the rocpd SQLite database) and lists calls,
mean/min duration and share per kernel.  ``cycle`` reads the per-launch ``*_kernel_trace.csv`` of a run of
``profile_kernels --solves K`` and splits the last complete V-cycle of the
last solve (from one residual norm to the next) by level: the descent
enters a coarser level after each restriction, the ascent a finer one at
each fused step that applies the coarse-grid correction.  ``pmc`` reads two
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs (``*_counter_collection.csv``)
of the same program, averages each counter (KiB per dispatch) over the
dispatches of the measured kernel and of the calibration copy kernel, and
scales the measured kernel's figures by known-bytes / counter of the copy
(8 bytes read and 8 written per cell).  The last line of its output is a
machine-readable record, tagged with a hash of the kernel sources, that the
benchmark reads to fill its HBM traffic field.
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/kernels.hpp", "csrc/vcycle_kernels.hpp")


def source_hash():
    """SHA-256 over the device-code sources (counters go stale when it changes)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name):
    return name.split("(")[0].replace("void ", "").strip()


def trace_rows(path):
    """[(kernel, calls, total_ns, avg_ns, min_ns)] from a stats csv or rocpd db."""
    rows = []
    if path.endswith(".csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append((short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]),
                             float(r["AverageNs"]), float(r["MinNs"])))
        return rows
    c = sqlite3.connect(path)
    acc = collections.defaultdict(list)
    for name, dur in c.execute("select name, duration from kernels"):
        acc[short(name)].append(dur)
    for k, v in acc.items():
        rows.append((k, len(v), float(sum(v)), sum(v) / len(v), float(min(v))))
    return rows


def cmd_trace(args):
    rows = sorted(trace_rows(args.path), key=lambda r: -r[2])
    tot = sum(r[2] for r in rows)
    print("total kernel time %.3f ms over %d launches\n" % (tot / 1e6, sum(r[1] for r in rows)))
    print("| kernel | calls | avg us | min us | total ms | share |")
    print("|---|---|---|---|---|---|")
    for k, n, t, a, m in rows:
        print("| `%s` | %d | %.2f | %.2f | %.3f | %.1f%% |" % (k, n, a / 1e3, m / 1e3, t / 1e6, 100 * t / tot))


def template_args(name):
    """['double', 'false', ...] of a demangled kernel name (empty if none)."""
    if "<" not in name:
        return []
    return [t.strip() for t in name[name.index("<") + 1:name.rindex(">")].split(",")]


def is_norm_launch(name):
    """A launch that yields a residual norm: the norm kernel, or a fused
    smoothing step instantiated with the norm flag (sixth template argument),
    which takes the norm of the iterate it starts from."""
    if name.startswith("k_resnorm"):
        return True
    ta = template_args(name)
    return name.startswith("k_smooth_fused") and len(ta) >= 6 and ta[5] == "true"


def is_correction_step(name):
    """The fused step that applies the coarse-grid correction (fifth
    template argument)."""
    ta = template_args(name)
    return name.startswith("k_smooth_fused") and len(ta) >= 5 and ta[4] == "true"


def cmd_cycle(args):
    with open(args.path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [short(r["Kernel_Name"]) for r in rows]
    st = [int(r["Start_Timestamp"]) for r in rows]
    en = [int(r["End_Timestamp"]) for r in rows]
    # the last solve: launches after the last idle gap longer than 300 us
    first = 0
    for i in range(1, len(rows)):
        if st[i] - en[i - 1] > 300000:
            first = i
    norms = [i for i in range(first, len(rows)) if is_norm_launch(names[i])]
    if len(norms) < 3:
        raise SystemExit("fewer than two complete cycles in the last solve")
    i0, i1 = norms[-3], norms[-2]
    level, lv_ns, lv_n, other, seq = 0, collections.defaultdict(float), collections.defaultdict(int), [], []
    for i in range(i0 + 1, i1 + 1):
        nm, d = names[i], en[i] - st[i]
        if is_correction_step(nm):
            level -= 1                      # ascent: the step that applies P e
        if nm.startswith(("k_smooth_fused", "k_restrict", "k_sweep", "k_smo2", "k_prolong")):
            lv_ns[level] += d
            lv_n[level] += 1
            seq.append((level, nm, d, st[i] - en[i - 1]))
        else:
            other.append((nm, d))
            seq.append(("", nm, d, st[i] - en[i - 1]))
        if nm.startswith("k_restrict"):
            level += 1                      # descent
    span = (en[i1] - en[i0]) / 1e3
    busy = sum(en[i] - st[i] for i in range(i0 + 1, i1 + 1)) / 1e3
    print("one V-cycle of the last solve: %.1f us from norm to norm, %.1f us in kernels, %d launches\n"
          % (span, busy, i1 - i0))
    print("(a cycle runs from one launch that yields a residual norm to the next: the norm kernel, or\n"
          "the next cycle's first fused step when that step takes the norm)\n")
    print("| level | launches | kernel time us | share of cycle |")
    print("|---|---|---|---|")
    for m in sorted(lv_ns):
        print("| %d | %d | %.1f | %.1f%% |" % (m, lv_n[m], lv_ns[m] / 1e3, 100 * lv_ns[m] / 1e3 / span))
    for nm, d in other:
        print("| `%s` | 1 | %.1f | %.1f%% |" % (nm, d / 1e3, 100 * d / 1e3 / span))
    print("| between launches | | %.1f | %.1f%% |" % (span - busy, 100 * (span - busy) / span))
    print("\nThe launches of that cycle in order (gap: from the previous launch's end to this one's start):\n")
    print("| # | level | kernel | us | gap us |")
    print("|---|---|---|---|---|")
    for k, (lv, nm, d, gap) in enumerate(seq):
        print("| %d | %s | `%s` | %.1f | %.1f |" % (k + 1, lv, nm, d / 1e3, gap / 1e3))


def counter_means(path, counter):
    acc = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def cmd_pmc(args):
    fetch = counter_means(args.fetch, "FETCH_SIZE")
    write = counter_means(args.write, "WRITE_SIZE")
    known_kib = 8.0 * args.cells / 1024.0
    cf, cw = fetch[args.calib_kernel][0], write[args.calib_kernel][0]
    sf, sw = known_kib / cf, known_kib / cw
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |")
    print("|---|---|---|---|")
    for k in sorted(set(fetch) | set(write)):
        print("| `%s` | %d | %.1f | %.1f |" % (k, fetch.get(k, (0, 0))[1], fetch.get(k, (0, 0))[0],
                                               write.get(k, (0, 0))[0]))
    print("\ncalibration: `%s` over %d cells moves %.1f KiB each way; counter scale fetch %.4f, write %.4f"
          % (args.calib_kernel, args.cells, known_kib, sf, sw))
    # one record per --kernel
    for kern in args.kernel:
        kf, kw = fetch[kern][0], write[kern][0]
        traffic = (kf * sf + kw * sw) * 1024.0
        print("\n`%s`: HBM traffic %.1f MB per launch (fetch %.1f MB, write %.1f MB, scaled)"
              % (kern, traffic / 1e6, kf * sf * 1024 / 1e6, kw * sw * 1024 / 1e6))
        rec = {"kernel": kern, "cells": args.cells, "traffic_bytes_per_launch": traffic,
               "fetch_kib": kf, "write_kib": kw, "scale_fetch": sf, "scale_write": sw,
               "sources_sha256": source_hash()}
        print("\n<!-- traffic-record %s -->" % json.dumps(rec))


def cmd_counters(args):
    """Per-kernel mean of every counter in one or more counter-collection
    files (kernels whose short name contains --match)."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    names = []
    for path in args.paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                k = short(r["Kernel_Name"])
                if args.match and args.match not in k:
                    continue
                c = r["Counter_Name"]
                if c not in names:
                    names.append(c)
                acc[k][c].append(float(r["Counter_Value"]))
    print("| kernel | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    for k in sorted(acc):
        vals = []
        for c in names:
            v = acc[k].get(c)
            vals.append("%.4g" % (sum(v) / len(v)) if v else "")
        print("| `%s` | %s |" % (k, " | ".join(vals)))


def read_traffic_record(md_path, kernel=None):
    """The record ``pmc`` wrote for kernel (the first one if kernel is None),
    or None if absent or the sources changed since."""
    try:
        with open(md_path) as f:
            for line in f:
                if line.startswith("<!-- traffic-record "):
                    rec = json.loads(line[len("<!-- traffic-record "):].rsplit("-->", 1)[0])
                    if kernel is not None and rec.get("kernel") != kernel:
                        continue
                    return rec if rec.get("sources_sha256") == source_hash() else None
    except OSError:
        return None
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("path")
    c = sub.add_parser("cycle")
    c.add_argument("path")
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("--cells", type=int, required=True)
    p.add_argument("--kernel", required=True, action="append",
                   help="kernel whose traffic record is written (repeatable)")
    p.add_argument("--calib-kernel", default="k_copy")
    q = sub.add_parser("counters")
    q.add_argument("paths", nargs="+")
    q.add_argument("--match", default="")
    args = ap.parse_args()
    {"trace": cmd_trace, "cycle": cmd_cycle, "pmc": cmd_pmc, "counters": cmd_counters}[args.cmd](args)


if __name__ == "__main__":
    main()
