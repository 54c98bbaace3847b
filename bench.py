#!/usr/bin/env python
"""Benchmark of the cut-cell multigrid solve on one MI355X.

Workload (the metric's configuration): unit square minus 3 seeded circles
(radii in [0.05, 0.15]), 2048^2 cells, Poisson (a, b, c) = (1, 0, 1),
Dirichlet data, manufactured u = sin(pi x) sin(pi y).  One step = one solve
of L u = f - N g from a zero guess until the relative L-infinity residual
(FP64, difference form) is <= 1e-10: boundary term, every V-cycle (sweeps,
SMO-2 blocks, restriction, prolongation, coarsest solve) and every residual
check.  Inputs are device-resident before timing; set-up is reported
separately.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METHOD_BYTES_PER_CELL = 24   # one FP64 smoothing sweep: read u and f-hat, write u'
METHOD_BYTES_PER_NNZ = 12    # a least-squares row entry: int32 column + FP64 weight


def method_step_bytes(n_cells, n_irr):
    """Algorithmic bytes of one FP64 smoothing step, counted as the method's
    own traffic: every cell's u and right-hand side read and its new value
    written (24 B), plus the 15-entry least-squares rows of the irregular
    cells (12 B per entry).  The SMO-2 block data (dense block inverses,
    overlapped rows) belong to this solver's smoother design, not to the
    method, and are reported separately (smo2_block_bytes)."""
    return METHOD_BYTES_PER_CELL * n_cells + METHOD_BYTES_PER_NNZ * 15 * n_irr


def smo2_block_bytes(st):
    """Bytes the SMO-2 blocks of one fused step move besides the method's
    own: their dense inverses, their overlapped rows' ELL entries (column
    4 B + weight 8 B) and per overlapped row its index, cell, row pointer,
    boundary-term index (4 B each), row sum, right-hand side and current
    value (8 B each), and the compact copy of their own rows (8 B)."""
    return st["inv_bytes"] + 12 * st["ext_nnz"] + 40 * st["ext_rows"] + 8 * st["rows"]


def sweep_bytes(n_cells):
    """One FP64 SMO-1 sweep (unfused schedule): 24 B per cell plus the kind
    byte."""
    return (METHOD_BYTES_PER_CELL + 1) * n_cells


def make_inputs(S, cfg, torch, dev):
    """f-hat and g-hat from the library's quadrature export (no oracle)."""
    import numpy as np

    grid = cfg["grid"]
    n, h = grid["nx"], grid["h"]
    sol = cfg["solution"]
    f = cfg["f"]
    # pure cells: 6x6 tensor Gauss-Legendre (host, row chunks)
    t, w = np.polynomial.legendre.leggauss(6)
    w2 = 0.25 * w[:, None] * w[None, :]
    xs = grid["x0"] + (np.arange(n)[None, :, None, None] + 0.5 + 0.5 * t[None, None, :, None]) * h

    def tensor_avg(fn):
        out = np.zeros((n, n))
        rows = max(1, (1 << 22) // (n * 36))
        for j0 in range(0, n, rows):
            j1 = min(n, j0 + rows)
            ys = grid["y0"] + (np.arange(j0, j1)[:, None, None, None] + 0.5 + 0.5 * t[None, None, None, :]) * h
            out[j0:j1] = (fn(xs, ys) * w2[None, None]).sum(axis=(2, 3))
        return out.ravel()

    fh = tensor_avg(f)
    ex = tensor_avg(sol.u)
    kinds, _ = S.kinds(0)
    vol = S.volumes(0)
    cell, qx, qy, qw = S.cell_quadrature()
    cut_sum = np.bincount(cell, weights=qw * f(qx, qy), minlength=n * n)
    cut = np.unique(cell)
    fh[cut] = cut_sum[cut] / vol[cut]
    fh[kinds <= 1] = 0.0
    fcell, fx, fy, fw, fnx, fny = S.face_quadrature()
    nf = S.info["n_bdry_faces"]
    _, fcurve, _ = S.boundary_faces()
    # the datum N u of each node's curve (u, du/dn or the Robin combination;
    # n is the outward normal of the domain)
    qcurve = fcurve[fcell]
    gv = np.zeros_like(fx)
    for ci, cu in enumerate(cfg["curves"]):
        m = qcurve == ci
        if np.any(m):
            gv[m] = sol.datum(cu, fx[m], fy[m], fnx[m], fny[m])
    ghat = np.bincount(fcell, weights=fw * gv, minlength=nf) / np.bincount(fcell, weights=fw, minlength=nf)
    ex[kinds <= 1] = 0.0
    ex[cut] = np.bincount(cell, weights=qw * sol.u(qx, qy), minlength=n * n)[cut] / vol[cut]
    return torch.tensor(fh, device=dev), torch.tensor(ghat, device=dev), ex, kinds


WORKLOADS = {
    4: "unit square minus 3 seeded circles (seed 4), %d^2 cells, Poisson, Dirichlet, u = sin(pi x) sin(pi y), "
       "FP64 V-cycles from zero to 1e-10",
    2: "unit square minus flower r = 0.25 + 0.05 sin 5t, %d^2 cells, (a,b,c) = (1,0.5,1), Dirichlet box, "
       "Neumann flower, u = exp(x) cos(3y), FP64 V-cycles from zero to 1e-10",
    5: "unit square minus 5 seeded ellipses (seed 5), %d^2 cells, (a,b,c) = (1,1.2,1), Dirichlet, "
       "u = sin(pi x) sin(2 pi y) + x^3, FP64 V-cycles from zero to 1e-10",
}


def run_error_study(args):
    """Discretization error of the FP64 solution on a sequence of grids
    (L-infinity over non-empty cells, volume-weighted L1 and L2), with the
    observed convergence rates.  The solves run to the rounding floor (tol
    1e-15, stopped by stagnation): at 1e-10 the iteration error, not the
    discretization error, would dominate on fine grids."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2504_00724_amd.ccgmg import Solver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for n in [int(v) for v in args.error_study.split(",")]:
        cfg = W.problem(args.problem, n) if args.problem else W.config(args.config, n=n)
        S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-15, max_cycles=80,
                   hip_stream=stream.cuda_stream)
        f, g, exact, kinds = make_inputs(S, cfg, torch, dev)
        S.set_boundary(g, 1)
        u = torch.zeros_like(f)
        rep = S.solve(f, u, raise_on_noconv=False)
        torch.cuda.synchronize()
        e = np.abs(u.cpu().numpy() - exact)
        ne = kinds >= 2
        vol = S.volumes(0)
        # L-infinity over non-empty cells; L1 and L2 weighted by the cut-cell
        # volumes and normalised by the domain's area
        w = vol[ne] / np.sum(vol[ne])
        row = {"n": n, "unknowns": S.info["n_unknowns"], "err_inf": float(np.max(e[ne])),
               "err_l1": float(np.sum(w * e[ne])), "err_l2": float(np.sqrt(np.sum(w * e[ne] ** 2))),
               "cycles": rep["cycles"], "rel_res_floor": rep["rel_res_inf"],
               "levels": S.info["n_levels"]}
        rows.append(row)
        print("error study n=%d: %s" % (n, row), file=sys.stderr, flush=True)
        S.close()
    for a, b in zip(rows, rows[1:]):
        b["rate_inf"] = float(np.log2(a["err_inf"] / b["err_inf"]))
        b["rate_l1"] = float(np.log2(a["err_l1"] / b["err_l1"]))
        b["rate_l2"] = float(np.log2(a["err_l2"] / b["err_l2"]))
    name = ("problem " + args.problem) if args.problem else WORKLOADS[args.config] % 0
    print(json.dumps({"error_study": name, "rows": rows}))


def fourier_averages(S, cfg, coeffs, torch, dev):
    """Cell averages of f = sum c_pq sin(p pi x) sin(q pi y): pure cells in
    closed form (the average of a product of sines over a square cell is the
    product of the one-dimensional averages), cut cells by the library's
    quadrature; zero on empty and merged cells."""
    import numpy as np
    grid = cfg["grid"]
    n, h = grid["nx"], grid["h"]
    m = coeffs.shape[0]
    k = np.arange(1, m + 1)[:, None] * np.pi
    xl = grid["x0"] + np.arange(n)[None, :] * h
    yl = grid["y0"] + np.arange(n)[None, :] * h
    sx = (np.cos(k * xl) - np.cos(k * (xl + h))) / (k * h)      # [p][i]
    sy = (np.cos(k * yl) - np.cos(k * (yl + h))) / (k * h)      # [q][j]
    fh = (sy.T @ coeffs.T @ sx).ravel()                          # [j][i]
    kinds, _ = S.kinds(0)
    vol = S.volumes(0)
    cell, qx, qy, qw = S.cell_quadrature()
    fx = np.zeros_like(qx)
    for p in range(m):
        for q in range(m):
            fx += coeffs[p, q] * np.sin((p + 1) * np.pi * qx) * np.sin((q + 1) * np.pi * qy)
    cut = np.unique(cell)
    fh[cut] = np.bincount(cell, weights=qw * fx, minlength=n * n)[cut] / vol[cut]
    fh[kinds <= 1] = 0.0
    return fh


def run_batch(args):
    """Batched workload: 64 right-hand sides (seeded Fourier sums, 8 x 8
    modes) on the unit square minus a disk r = 0.2 at 512^2, plus 32
    geometries with n in {128, 256, 512, 1024} and 1-3 seeded ellipse holes,
    homogeneous Dirichlet data, all solved together by one captured
    multi-branch launch per V-cycle."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2504_00724_amd.ccgmg import Batch, Solver
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    prec = 0 if args.batch_fp64 else 1
    from paper_2504_00724_amd.ccgmg import create_many
    t0 = time.perf_counter()
    probs = [W.config(3, n=512)] + W.batch_geometries(args.batch_geometries)
    sched = {} if args.batch_tune else dict(tune_schedule=0, smoother_fused=1, nu1=args.batch_nu, nu2=args.batch_nu,
                                            smo2_every_sweep=args.batch_smo2_every, omega=args.batch_omega)
    opts = [dict(tol=1e-10, max_cycles=200, hip_stream=stream, max_nrhs=(args.batch_rhs if i == 0 else 1),
                 precision=prec, **sched) for i in range(len(probs))]
    problems = [(c["grid"], c["curves"], c["a"], c["b"], c["c"]) for c in probs]
    if args.batch_setup == "many":
        # host set-up of all geometries concurrently, device set-up as each is ready
        solvers = create_many(problems, opts)
    else:
        solvers = [Solver(*p, **o) for p, o in zip(problems, opts)]
    setup_s = time.perf_counter() - t0
    fs, us, nr, nu = [], [], [], 0
    for i, (cfg, S) in enumerate(zip(probs, solvers)):
        m = args.batch_rhs if i == 0 else 1
        seeds = [3000 + z for z in range(m)] if i == 0 else [3000 + i - 1]
        F = np.stack([fourier_averages(S, cfg, W.fourier_rhs(sd)[1], torch, dev) for sd in seeds])
        fs.append(torch.tensor(F, device=dev))
        us.append(torch.zeros_like(fs[-1]))
        nr.append(m)
        nu += S.info["n_unknowns"] * m
        print("geometry %d: n=%d unknowns %d x %d rhs, levels %d, library set-up %.1f s" % (
            i, cfg["grid"]["nx"], S.info["n_unknowns"], m, S.info["n_levels"], S.info["setup_seconds"]),
            file=sys.stderr, flush=True)
    print("batch set-up (%s): %.1f s" % (args.batch_setup, setup_s), file=sys.stderr, flush=True)
    B = Batch(solvers, nbranches=args.batch_branches)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        B.solve(fs, us, nr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        reps = B.solve(fs, us, nr)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t1) / args.steps
    # the same problems solved one after another (same contexts)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for S, f, u, m in zip(solvers, fs, us, nr):
        S.solve(f, u, m)
    torch.cuda.synchronize()
    seq_ms = 1e3 * (time.perf_counter() - t2)
    out = {
        "metric": "batched cut-cell GMG solve: unknowns x right-hand sides per second at 1e-10 rel. residual",
        "value": nu / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec else "f64", "data": "synthetic",
        "config": {"workload": "%d RHS on unit square minus disk r=0.2 at 512^2 + %d seeded ellipse geometries, "
                               "n in {128,256,512,1024}, homogeneous Dirichlet, Fourier RHS 8x8 modes"
                               % (args.batch_rhs, args.batch_geometries),
                   "unknowns_x_rhs": nu, "branches": args.batch_branches,
                   "schedule": "tuned per context" if args.batch_tune else
                               "%d + %d fused steps, SMO-2 in every %d. step, SMO-1 weight %.2f"
                               % (args.batch_nu, args.batch_nu, args.batch_smo2_every, args.batch_omega),
                   "precision": "FP32 V-cycles in FP64 refinement" if prec else "FP64"},
        "max_cycles": max(r["cycles"] for r in reps), "worst_rel_res": max(r["rel_res_inf"] for r in reps),
        "sequential_ms": seq_ms, "speedup_vs_sequential": seq_ms / ms, "setup_s": setup_s,
        "setup_mode": "ccgmg_create_many (concurrent host set-up)" if args.batch_setup == "many"
                      else "ccgmg_create one geometry after another",
    }
    print(json.dumps(out))
    B.close()
    for S in solvers:
        S.close()


def _cpu_worker(conn, n_sample, seconds, config, threads):
    """Child process of the CPU baseline: the oracle's set-up (untimed) runs
    while the parent measures the GPU; on the parent's signal the oracle's
    own V-cycle solve (Alg. 2, exact SMO-2, LU at the coarsest level) from a
    zero guess is repeated for at least ``seconds`` on 1 thread, then on
    ``threads`` threads."""
    try:
        from threadpoolctl import threadpool_limits

        import workloads as W
        from oracle.discretization import boundary_data
        from oracle.geometry import cell_averages
        from oracle.multigrid import Hierarchy, rhs_vector
        cfg = W.config(config, n=n_sample)
        t_set = time.perf_counter()
        with threadpool_limits(limits=threads):
            H = Hierarchy(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
            H.select_depth()
            lv = H.levels[0]
            f = cell_averages(lv.cg, cfg["f"]).ravel()
            g = boundary_data(lv.disc, cfg["solution"])
            r = rhs_vector(lv, f, g)
        t_set = time.perf_counter() - t_set
        conn.send(("ready", t_set))
        if conn.recv() != "go":
            return
        runs = {}
        for nt in (1, threads):
            with threadpool_limits(limits=nt):
                solves, cycles = 0, 0
                t0 = time.perf_counter()
                while True:
                    hist = []
                    H.solve(r, tol=1e-10, history=hist)
                    solves += 1
                    cycles = len(hist)
                    dt = time.perf_counter() - t0
                    if dt >= seconds:
                        break
            runs[nt] = (solves, dt, cycles)
        conn.send(("done", {"runs": runs, "unknowns": int(lv.nonempty.sum()), "setup_s": t_set}))
    except Exception as e:   # reported by the parent, never raised into the GPU run
        conn.send(("error", repr(e)))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class CpuBaseline:
    """The oracle timed on the host cores beside the GPU run, in a child
    process started before the GPU is touched."""

    def __init__(self, n_sample, seconds, config):
        import multiprocessing as mp
        self.n, self.seconds = n_sample, seconds
        # the machine's CPU share for one GPU is given by OMP_NUM_THREADS there
        self.threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        ctx = mp.get_context("spawn")
        self.conn, child = ctx.Pipe()
        self.proc = ctx.Process(target=_cpu_worker, args=(child, n_sample, seconds, config, self.threads),
                                daemon=True)
        self.proc.start()

    def result(self, timeout=900.0):
        """Waits for the set-up, starts the timed solves and returns the
        cpu_baseline record (None if the child failed)."""
        try:
            if not self.conn.poll(timeout):
                return None
            tag, t_set = self.conn.recv()
            if tag != "ready":
                print("cpu baseline failed: %s" % t_set, file=sys.stderr, flush=True)
                return None
            self.conn.send("go")
            if not self.conn.poll(timeout):
                return None
            tag, res = self.conn.recv()
            if tag != "done":
                print("cpu baseline failed: %s" % res, file=sys.stderr, flush=True)
                return None
        finally:
            self.proc.join(timeout=5)
        nu = res["unknowns"]
        (s1, d1, c1), (sn, dn, cn) = res["runs"][1], res["runs"][self.threads]
        affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
        return {"value": nu * sn / dn, "unit": "unknowns/s", "cores": self.threads, "kind": "oracle",
                "sample": "oracle V-cycle solves (Alg. 2, exact SMO-2 blocks, LU at the coarsest level) from zero "
                          "to 1e-10 on the same geometry and problem at %d^2 (%d unknowns, %d cycles per solve): "
                          "%d solves in %.1f s with %d threads allowed (%d solves in %.1f s on 1 thread); oracle "
                          "set-up %.1f s untimed, run while the GPU was measured"
                          % (self.n, nu, cn, sn, dn, self.threads, s1, d1, res["setup_s"]),
                "config": {"grid": self.n, "unknowns": nu, "cycles_per_solve": cn},
                "single_core": {"value": nu * s1 / d1, "solves": s1, "seconds": d1},
                "nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="grid side (default: the workload's own)")
    ap.add_argument("--config", type=int, choices=[2, 4, 5], default=4,
                    help="4: the metric workload; 2: flower hole with Neumann data, b = 0.5 (1024^2); "
                         "5: five ellipses, b = 1.2 (4096^2)")
    ap.add_argument("--error-study", default="",
                    help="comma-separated grid sides: FP64 solves of the chosen workload and their errors")
    ap.add_argument("--problem", choices=["P1", "P2N", "P2D", "P3"], default="",
                    help="with --error-study: one of the paper's test problems instead of a workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=512)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-fmg", action="store_true", help="skip the FMG-cycle solve")
    ap.add_argument("--no-fp64-inverses", action="store_true",
                    help="skip the extra solve with FP64-stored SMO-2 and coarsest inverses")
    ap.add_argument("--prolongation", type=int, default=0)
    ap.add_argument("--smo2-every-sweep", type=int, default=1)
    ap.add_argument("--workload", choices=["metric", "batch"], default="metric",
                    help="metric: the three-circle Poisson solve at --n; batch: the batched workload")
    ap.add_argument("--batch-rhs", type=int, default=64)
    ap.add_argument("--batch-geometries", type=int, default=32)
    ap.add_argument("--batch-branches", type=int, default=4)
    ap.add_argument("--batch-fp64", action="store_true")
    ap.add_argument("--batch-nu", type=int, default=4,
                    help="batched workload: fused smoothing steps before and after the coarse correction")
    ap.add_argument("--batch-smo2-every", type=int, default=3,
                    help="batched workload: SMO-2 in every s-th of the fused steps (1: every step)")
    ap.add_argument("--batch-omega", type=float, default=0.7,
                    help="batched workload: SMO-1 weight (the paper's experiments use 0.5)")
    ap.add_argument("--batch-setup", choices=["many", "one"], default="many",
                    help="many: ccgmg_create_many (concurrent host set-up); one: ccgmg_create per geometry")
    ap.add_argument("--batch-tune", type=int, default=0,
                    help="1: every batch context tunes its own smoothing schedule (slower set-up)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if not args.n:
        args.n = {2: 1024, 4: 2048, 5: 4096}[args.config]
    if args.error_study:
        run_error_study(args)
        return
    # the oracle's set-up overlaps the GPU measurement (child process,
    # started before the GPU is touched)
    cpu_job = None if args.no_cpu_baseline else CpuBaseline(args.cpu_sample_n, args.cpu_seconds, args.config)

    import numpy as np
    import torch

    import workloads as W
    from paper_2504_00724_amd.ccgmg import Solver
    from paper_2504_00724_amd.prof_summary import read_traffic_record

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    cfg = W.config(args.config, n=args.n)
    t0 = time.perf_counter()
    S = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
               hip_stream=stream.cuda_stream, prolongation=args.prolongation,
               smo2_every_sweep=args.smo2_every_sweep)
    setup_s = time.perf_counter() - t0
    info = S.info
    print("set-up %.1f s: %s" % (setup_s, info), file=sys.stderr, flush=True)
    f, g, exact, kinds = make_inputs(S, cfg, torch, dev)
    S.set_boundary(g, 1)
    # set-up, untimed: schedule and depth re-chosen on this problem
    t1 = time.perf_counter()
    S.tune(f)
    setup_s += time.perf_counter() - t1
    info = S.info
    print("tuned on the workload: %s" % info, file=sys.stderr, flush=True)
    u = torch.zeros_like(f)
    torch.cuda.synchronize()

    def run(solver, uu, steps, walls=None):
        reps = []
        for _ in range(steps):
            a = time.perf_counter()
            reps.append(solver.solve(f, uu))   # returns once the solve has finished on the device
            if walls is not None:
                walls.append(1e3 * (time.perf_counter() - a))
        return reps

    run(S, u, args.warmup)
    torch.cuda.synchronize()
    walls = []
    t0 = time.perf_counter()
    reps = run(S, u, args.steps, walls)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / args.steps
    nu = info["n_unknowns"]
    devs = [1e3 * r["seconds"] for r in reps]
    per_solve = {"wall_ms_mean": float(np.mean(walls)), "wall_ms_median": float(np.median(walls)),
                 "wall_ms_max": float(np.max(walls)), "device_ms_mean": float(np.mean(devs)),
                 "device_ms_median": float(np.median(devs)), "device_ms_max": float(np.max(devs))}
    # relative L2 residual of the final iterate (after the timed region)
    res_l2 = S.residual_norms(f, u)[1][0]
    u64 = u.cpu().numpy()
    ne = kinds >= 2
    disc_err = float(np.max(np.abs(u64 - exact)[ne]))

    # dominant kernel: the finest-level smoothing step (fused SMO-1 + SMO-2
    # launch, or the SMO-1 sweep of the unfused schedule), timed with HIP
    # events on the library's stream right after the timed solves
    ty = S.tuning(0)[0]
    cells = args.n * args.n
    block_bytes = 0
    if info["smoother_fused"]:
        kname = "k_smooth_fused<double, %s, true, %d, false, false>" % ("true" if cfg["b"] != 0 else "false", ty)
        kdesc = "finest-level fused SMO-1 + SMO-2 step"
        dom_us = S.profile_kernel(7, 0, 50)
        dom_bytes = method_step_bytes(cells, info["n_irregular"])
        block_bytes = smo2_block_bytes(S.smo2_stats(0))
    else:
        kname = "k_sweep<double, %s, true, %d>" % ("true" if cfg["b"] != 0 else "false", ty)
        kdesc = "finest-level SMO-1 sweep"
        dom_us = S.profile_kernel(0, 0, 50)
        dom_bytes = sweep_bytes(cells)
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    other = {name: S.profile_kernel(k, 0, 20) for name, k in (("sweep_us", 0), ("restrict_us", 1),
                                                               ("prolong_us", 2), ("smo2_block_us", 3),
                                                               ("copy_us", 6))}
    # measured bandwidth ceiling: a plain FP64 copy of one finest-level array
    copy_gbs = 16.0 * cells / (other["copy_us"] * 1e-6) / 1e9

    # HBM bytes per launch of the same kernel from the committed counter runs
    # (FETCH_SIZE, WRITE_SIZE, copy-calibrated); null once the kernel sources
    # differ from those the counters were taken on
    rec = read_traffic_record(os.path.join(ROOT, "profiles", "smoothing_step_fp64_2048_pmc.md"), kname)
    traffic = None
    if rec and rec["cells"] == cells and rec["kernel"] == kname:
        traffic = rec["traffic_bytes_per_launch"]

    tiles = [S.tuning(m)[0] for m in range(info["n_levels"])]

    # the same solve with both dense inverses (SMO-2 blocks, coarsest level)
    # stored in FP64 rather than FP32
    fp64_inv = None
    if not args.no_fp64_inverses:
        S64 = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
                     hip_stream=stream.cuda_stream, prolongation=args.prolongation,
                     smo2_every_sweep=args.smo2_every_sweep, inverse_fp32=0)
        S64.set_boundary(g, 1)
        S64.tune(f)
        u2 = torch.zeros_like(f)
        run(S64, u2, args.warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r64 = run(S64, u2, args.steps)
        torch.cuda.synchronize()
        m64 = 1e3 * (time.perf_counter() - t1) / args.steps
        fp64_inv = {"value": nu / (m64 * 1e-3), "ms_per_step": m64, "cycles": r64[-1]["cycles"],
                    "rel_res_inf": r64[-1]["rel_res_inf"],
                    "device_ms_median": 1e3 * float(np.median([r["seconds"] for r in r64])),
                    "schedule": {k: S64.info[k] for k in ("nu1", "nu2", "nu1_coarse", "nu2_coarse", "smo2_every_sweep",
                                                                   "omega")}}
        S64.close()
        del u2

    mixed = None
    if not args.no_mixed:
        Sm = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
                    hip_stream=stream.cuda_stream, precision=1, prolongation=args.prolongation,
                    smo2_every_sweep=args.smo2_every_sweep)
        Sm.set_boundary(g, 1)
        Sm.tune(f)
        um = torch.zeros_like(f)
        for _ in range(args.warmup):
            Sm.solve(f, um)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            rm = Sm.solve(f, um)
        torch.cuda.synchronize()
        mms = 1e3 * (time.perf_counter() - t1) / args.steps
        diff = float(np.max(np.abs(um.cpu().numpy() - u64)[ne]) / np.max(np.abs(u64[ne])))
        mixed = {"value": nu / (mms * 1e-3), "ms_per_step": mms, "cycles": rm["cycles"],
                 "rel_res_inf": rm["rel_res_inf"], "rel_diff_vs_fp64": diff,
                 "disc_err_inf": float(np.max(np.abs(um.cpu().numpy() - exact)[ne]))}
        Sm.close()

    # the same problem by FMG cycles (Section 4, Fig. FMG-cycle), tuned the
    # same way
    fmg = None
    if not args.no_fmg:
        Sf = Solver(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], tol=1e-10, max_cycles=200,
                    hip_stream=stream.cuda_stream, cycle=1)
        Sf.set_boundary(g, 1)
        Sf.tune(f)
        uf = torch.zeros_like(f)
        run(Sf, uf, args.warmup)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rf = run(Sf, uf, args.steps)
        torch.cuda.synchronize()
        mf = 1e3 * (time.perf_counter() - t1) / args.steps
        fmg = {"value": nu / (mf * 1e-3), "ms_per_step": mf, "cycles": rf[-1]["cycles"],
               "rel_res_inf": rf[-1]["rel_res_inf"],
               "rel_diff_vs_fp64": float(np.max(np.abs(uf.cpu().numpy() - u64)[ne]) / np.max(np.abs(u64[ne]))),
               "schedule": {k: Sf.info[k] for k in ("nu1", "nu2", "nu1_coarse", "nu2_coarse", "smo2_every_sweep", "n_levels",
                                                     "omega")}}
        Sf.close()

    cpu = cpu_job.result() if cpu_job else None

    out = {
        "metric": ("4th-order cut-cell GMG solve: unknowns/s and HBM GB/s at 1e-10 rel. residual, 2048^2"
                   if args.config == 4 else "4th-order cut-cell GMG solve: unknowns/s at 1e-10 rel. residual"),
        "value": nu / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config] % args.n,
                   "n_unknowns": nu, "n_irregular": info["n_irregular"], "levels": info["n_levels"],
                   "coarsest": info["nx_coarsest"], "nrhs": 1,
                   "schedule": {"smoother_fused": info["smoother_fused"], "nu1": info["nu1"], "nu2": info["nu2"],
                                "nu1_coarse": info["nu1_coarse"], "nu2_coarse": info["nu2_coarse"],
                                "smo2_every_sweep": info["smo2_every_sweep"], "omega": info["omega"]},
                   "sweep_tile_rows": tiles,
                   # dense inverses are computed in FP64 and applied in FP64
                   # arithmetic; this is their storage (fp64_inverses below:
                   # the same solve with both stored in FP64)
                   "inverse_storage": {"smo2_blocks": "fp32", "coarsest": "fp32"}},
        "cycles": reps[-1]["cycles"],
        "rel_res_inf": reps[-1]["rel_res_inf"],
        "rel_res_l2": res_l2,
        "ms_median_device": per_solve["device_ms_median"],
        "per_solve": per_solve,
        "disc_err_inf": disc_err,
        "setup_s": setup_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "%s (%s)" % (kname, kdesc), "avg_us": dom_us,
                     "alg_bytes_per_launch": dom_bytes,
                     "alg_bytes_rule": "24 B per cell (u, f read; u' written) + 12 B per least-squares entry",
                     "smo2_block_bytes_per_launch": block_bytes,
                     "traffic_over_alg": (traffic / dom_bytes) if traffic else None,
                     "traffic_unit": "bytes per launch",
                     "copy_ceiling_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "kernels_us": other,
        "fp64_inverses": fp64_inv,
        "mixed_precision": mixed,
        "fmg": fmg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    S.close()


if __name__ == "__main__":
    main()
