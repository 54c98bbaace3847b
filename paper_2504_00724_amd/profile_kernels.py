"""Launch single V-cycle kernels on the finest level of the three-circle
Poisson workload (unit square minus 3 seeded circles, n^2 cells), for
hardware-counter collection under a profiler, e.g.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- \
        python3 -m paper_2504_00724_amd.profile_kernels --n 2048

Kernel 0 is the FP64 SMO-1 sweep, kernel 8 two sweeps in one launch, kernel
6 a plain FP64 copy of the same
cell array (16 bytes per cell), which calibrates the byte counters.

With --solves K it instead builds the context as the benchmark does (tuned
tiles, schedule and depth) and runs K FP64 solves of the benchmark's problem
to 1e-10, for a per-launch kernel trace of whole V-cycles.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

KERNELS = {"sweep": 0, "restrict": 1, "prolong": 2, "smo2": 3, "sweep_f32": 5, "copy": 6, "fused": 7, "sweep2": 8,
           "fused_pro": 9, "fused_norm_host": 10, "fused_norm_dev": 11}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--kernels", default="sweep,copy")
    ap.add_argument("--tile-rows", default="32",
                    help="SMO-1 tile heights, comma-separated (8, 16, 32): the kernels are launched "
                         "for each (the benchmark tunes its finest level among them)")
    ap.add_argument("--solves", type=int, default=0)
    ap.add_argument("--config", type=int, choices=[2, 4, 5], default=4,
                    help="workload: 4 three circles (b = 0), 5 five ellipses (b = 1.2), 2 flower (b = 0.5)")
    args = ap.parse_args()
    import torch  # noqa: F401  (HIP runtime and device selection)

    import workloads as W
    from paper_2504_00724_amd.ccgmg import Solver
    cfg = W.config(args.config, n=args.n)
    if args.solves:
        import bench
        dev = torch.device("cuda:0")
        S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
                   hip_stream=torch.cuda.current_stream().cuda_stream)
        f, g, _, _ = bench.make_inputs(S, cfg, torch, dev)
        S.set_boundary(g, 1)
        S.tune(f)
        for k in range(args.solves):
            u = torch.zeros_like(f)
            torch.cuda.synchronize()
            time.sleep(0.01)   # an idle gap that marks the solve in the trace
            rep = S.solve(f, u)
            torch.cuda.synchronize()
            print("solve %d: %d cycles, %.3f ms" % (k, rep["cycles"], 1e3 * rep["seconds"]), flush=True)
        S.close()
        return
    for ty in [int(t) for t in args.tile_rows.split(",")]:
        S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], auto_depth=0, sweep_tile_rows=ty)
        out = {"n": args.n, "cells": args.n * args.n, "tile_rows": ty}
        for name in args.kernels.split(","):
            out[name + "_us"] = S.profile_kernel(KERNELS[name], 0, args.reps)
            print(name, "done", flush=True)
        print(json.dumps(out), flush=True)
        S.close()


if __name__ == "__main__":
    main()
