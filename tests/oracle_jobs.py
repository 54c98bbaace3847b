"""Oracle computations that the GPU parity tests farm out to worker
processes.

The workers are started with the "spawn" method, so they are fresh
interpreters that never touch the GPU (the test process has initialised
HIP; a forked copy of it would inherit its device handles).  Each worker
keeps the geometry and discretization it built, keyed by the workload, so
that several chunks of rows cost one build per worker.  Nothing here is
imported by the library; only tests use it.
"""
from __future__ import annotations

import os

import numpy as np

_CACHE = {}


def _config(case, n):
    import workloads as W
    return W.problem(case, n) if isinstance(case, str) else W.config(case, n=n)


def _discretization(case, n):
    key = (case, n)
    if key not in _CACHE:
        from oracle.discretization import Discretization
        from oracle.geometry import CutGrid
        cfg = _config(case, n)
        cg = CutGrid(cfg["grid"], cfg["curves"])
        _CACHE[key] = Discretization(cg, cfg["a"], cfg["b"], cfg["c"], eager=False)
    return _CACHE[key]


def fit_rows(case, n, rows):
    """The oracle's least-squares rows of the given irregular cells: {q:
    (lattice cells, weights in 1/h^2 units, [(face index, weight)])}."""
    d = _discretization(case, n)
    out = {}
    for q in rows:
        cells, w, fw = d.row(int(q))
        out[int(q)] = (list(cells), np.asarray(w, dtype=float), list(fw))
    return out


def direct_reference(case, n):
    """Data and reference solution of a workload on one grid: the oracle's
    cell averages f-hat, face data g-hat, the direct solve of L u = f - N g
    and the non-empty mask."""
    from oracle.discretization import boundary_data
    from oracle.geometry import cell_averages
    from oracle.multigrid import Level, direct_solve, rhs_vector
    cfg = _config(case, n)
    lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
    f = cell_averages(lv.cg, cfg["f"]).ravel()
    g = boundary_data(lv.disc, cfg["solution"])
    ref = direct_solve(lv, rhs_vector(lv, f, g))
    return f, g, ref, np.asarray(lv.nonempty, dtype=bool)


def lattice_rule_p2n_error(rule, n):
    """L-infinity error of Problem 2 (Neumann data on the ellipse) at n^2
    with the given lattice rule of the oracle."""
    import workloads as W
    from oracle.discretization import boundary_data
    from oracle.geometry import cell_averages
    from oracle.multigrid import Level, direct_solve, rhs_vector
    from oracle.norms import norms
    cfg = W.problem2(n, hole_bc=W.NEUMANN)
    lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], lattice_rule=rule)
    f = cell_averages(lv.cg, cfg["f"])
    g = boundary_data(lv.disc, cfg["solution"])
    u = direct_solve(lv, rhs_vector(lv, f, g))
    return norms(u - cell_averages(lv.cg, cfg["solution"].u).ravel(), lv.cg.vol)[2]


def lattice_rule_vcycle_history(rule, k, n, cycles):
    """Relative residuals of the oracle's two-level V-cycles (zero start,
    seeded random right-hand side) on workload k at n^2 with the given
    lattice rule."""
    import numpy as np
    import workloads as W
    from oracle.multigrid import Hierarchy
    cfg = W.config(k, n=n)
    H = Hierarchy(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"], lattice_rule=rule, max_levels=2)
    r = np.random.default_rng(5).standard_normal(n * n) * H.levels[0].nonempty
    hist = []
    H.solve(r, tol=1e-10, max_cycles=cycles, history=hist)
    return hist


def pool(workers=None):
    """A process pool of fresh interpreters, sized to the host's CPU share
    (at most 8 workers)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    return ProcessPoolExecutor(max_workers=workers or max(1, min(8, share)), mp_context=mp.get_context("spawn"))


def all_rows(case, n, irregular, chunks=32):
    """fit_rows over every irregular cell, spread over a pool."""
    parts = np.array_split(np.asarray(irregular), chunks)
    out = {}
    with pool() as ex:
        for res in ex.map(fit_rows, [case] * len(parts), [n] * len(parts), [list(map(int, p)) for p in parts]):
            out.update(res)
    return out
