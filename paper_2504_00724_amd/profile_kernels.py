"""Launch single V-cycle kernels on the finest level of the three-circle
Poisson workload (unit square minus 3 seeded circles, n^2 cells), for
hardware-counter collection under a profiler, e.g.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- \
        python3 -m paper_2504_00724_amd.profile_kernels --n 2048

Kernel 0 is the FP64 SMO-1 sweep, kernel 6 a plain FP64 copy of the same
cell array (16 bytes per cell), which calibrates the byte counters.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

KERNELS = {"sweep": 0, "restrict": 1, "prolong": 2, "smo2": 3, "sweep_f32": 5, "copy": 6, "fused": 7}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--kernels", default="sweep,copy")
    ap.add_argument("--tile-rows", type=int, default=32,
                    help="SMO-1 tile height (the benchmark's tuned choice on the finest level)")
    args = ap.parse_args()
    import torch  # noqa: F401  (HIP runtime and device selection)

    import workloads as W
    from paper_2504_00724_amd.ccgmg import Solver
    cfg = W.config(4, n=args.n)
    S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], auto_depth=0,
               sweep_tile_rows=args.tile_rows)
    out = {"n": args.n, "cells": args.n * args.n}
    for name in args.kernels.split(","):
        out[name + "_us"] = S.profile_kernel(KERNELS[name], 0, args.reps)
        print(name, "done", flush=True)
    print(json.dumps(out), flush=True)
    S.close()


if __name__ == "__main__":
    main()
