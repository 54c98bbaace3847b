"""Summaries of rocprofv3 output as short Markdown tables.

    python3 -m paper_2504_00724_amd.prof_summary trace STATS.csv|RESULTS.db
    python3 -m paper_2504_00724_amd.prof_summary pmc FETCH.csv WRITE.csv \
        --cells N --kernel NAME [--calib-kernel k_copy]

``trace`` reads a ``--kernel-trace --stats`` run (the ``*_kernel_stats.csv``
of ``--output-format csv``, or the rocpd SQLite database) and lists calls,
mean/min duration and share per kernel.  ``pmc`` reads two
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
    kf, kw = fetch[args.kernel][0], write[args.kernel][0]
    traffic = (kf * sf + kw * sw) * 1024.0
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB |")
    print("|---|---|---|---|")
    for k in sorted(set(fetch) | set(write)):
        print("| `%s` | %d | %.1f | %.1f |" % (k, fetch.get(k, (0, 0))[1], fetch.get(k, (0, 0))[0],
                                               write.get(k, (0, 0))[0]))
    print("\ncalibration: `%s` over %d cells moves %.1f KiB each way; counter scale fetch %.4f, write %.4f"
          % (args.calib_kernel, args.cells, known_kib, sf, sw))
    print("\n`%s`: HBM traffic %.1f MB per launch (fetch %.1f MB, write %.1f MB, scaled)"
          % (args.kernel, traffic / 1e6, kf * sf * 1024 / 1e6, kw * sw * 1024 / 1e6))
    rec = {"kernel": args.kernel, "cells": args.cells, "traffic_bytes_per_launch": traffic,
           "fetch_kib": kf, "write_kib": kw, "scale_fetch": sf, "scale_write": sw,
           "sources_sha256": source_hash()}
    print("\n<!-- traffic-record %s -->" % json.dumps(rec))


def read_traffic_record(md_path):
    """The record written by ``pmc``, or None if absent or the sources changed."""
    try:
        with open(md_path) as f:
            for line in f:
                if line.startswith("<!-- traffic-record "):
                    rec = json.loads(line[len("<!-- traffic-record "):].rsplit("-->", 1)[0])
                    return rec if rec.get("sources_sha256") == source_hash() else None
    except OSError:
        return None
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("path")
    p = sub.add_parser("pmc")
    p.add_argument("fetch")
    p.add_argument("write")
    p.add_argument("--cells", type=int, required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--calib-kernel", default="k_copy")
    args = ap.parse_args()
    (cmd_trace if args.cmd == "trace" else cmd_pmc)(args)


if __name__ == "__main__":
    main()
