"""ctypes binding of libccgmg.so (the C interface in include/ccgmg.h).

Argument marshalling only: every step of the set-up and the solve runs in
the native library.  Device arrays are passed as raw pointers of torch CUDA
(HIP) tensors; torch supplies device memory and the stream.  The library
must be built (``paper_2504_00724_amd.build.build()``); loading fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccgmg.so")

OK, EINVAL, ENOTELLIPTIC, EGEOM, EPLG, ESINGULAR, ENOCONV, EDEVICE, ENOMEM = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTELLIPTIC", -3: "EGEOM", -4: "EPLG", -5: "ESINGULAR", -6: "ENOCONV",
          -7: "EDEVICE", -8: "ENOMEM"}

EXPORTS = ["ccgmg_default_options", "ccgmg_create", "ccgmg_create_many", "ccgmg_query", "ccgmg_get_cell_kinds", "ccgmg_get_level_shape",
           "ccgmg_get_volumes", "ccgmg_get_counts", "ccgmg_get_irregular", "ccgmg_get_stencils", "ccgmg_get_boundary_faces",
           "ccgmg_get_alg3_order", "ccgmg_cell_quadrature", "ccgmg_face_quadrature", "ccgmg_apply", "ccgmg_residual_norms",
           "ccgmg_residual_norms_noalloc",
           "ccgmg_set_boundary", "ccgmg_solve", "ccgmg_solve_adjoint", "ccgmg_apply_adjoint", "ccgmg_apply_NT",
           "ccgmg_profile_kernel", "ccgmg_get_tuning", "ccgmg_get_smo2_stats", "ccgmg_tune",
           "ccgmg_batch_create", "ccgmg_batch_solve", "ccgmg_batch_last_error", "ccgmg_batch_destroy",
           "ccgmg_last_error", "ccgmg_create_error", "ccgmg_destroy"]


class CurveT(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double * 8), ("domain_inside", C.c_int), ("bc", C.c_int),
                ("robin", C.c_double * 2)]


class GridT(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("h", C.c_double), ("nx", C.c_int), ("ny", C.c_int)]


class OptionsT(C.Structure):
    _fields_ = [("theta", C.c_double), ("w_min", C.c_double), ("omega", C.c_double), ("nu1", C.c_int),
                ("nu2", C.c_int), ("nu1_coarse", C.c_int), ("nu2_coarse", C.c_int), ("coarsest_min_n", C.c_int), ("max_levels", C.c_int), ("auto_depth", C.c_int),
                ("depth_max_rate", C.c_double), ("precision", C.c_int), ("prolongation", C.c_int),
                ("smo2_every_sweep", C.c_int), ("smo2_iters", C.c_int), ("smo2_block", C.c_int),
                ("smo2_overlap", C.c_int), ("smo2_widen", C.c_int), ("tol", C.c_double), ("max_cycles", C.c_int), ("max_nrhs", C.c_int),
                ("use_initial_guess", C.c_int), ("num_threads", C.c_int), ("use_graph", C.c_int),
                ("tune_tiles", C.c_int), ("sweep_tile_rows", C.c_int), ("smoother_fused", C.c_int), ("tune_schedule", C.c_int), ("inverse_fp32", C.c_int), ("host_only", C.c_int),
                ("cycle", C.c_int), ("tune_cache", C.c_int), ("hip_stream", C.c_void_p)]


class ProblemT(C.Structure):
    _fields_ = [("grid", GridT), ("curves", C.POINTER(CurveT)), ("ncurves", C.c_int), ("a", C.c_double),
                ("b", C.c_double), ("c", C.c_double)]


class InfoT(C.Structure):
    _fields_ = [("n_cells", C.c_long), ("n_unknowns", C.c_long), ("n_irregular", C.c_long),
                ("n_bdry_faces", C.c_long), ("n_levels", C.c_int), ("nx_coarsest", C.c_int),
                ("ny_coarsest", C.c_int), ("coarse_unknowns", C.c_long), ("setup_seconds", C.c_double),
                ("plg_max_cond", C.c_double), ("smoother_fused", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("nu1_coarse", C.c_int), ("nu2_coarse", C.c_int), ("smo2_every_sweep", C.c_int),
                ("omega", C.c_double)]


class ReportT(C.Structure):
    _fields_ = [("cycles", C.c_int), ("outer_iters", C.c_int), ("rel_res_inf", C.c_double),
                ("rel_res_2", C.c_double), ("seconds", C.c_double), ("history", C.c_double * 64)]


_LIB = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libccgmg.so is not built; run paper_2504_00724_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.c_int
        L.ccgmg_default_options.argtypes = [C.POINTER(OptionsT)]
        L.ccgmg_default_options.restype = None
        L.ccgmg_create.argtypes = [C.POINTER(GridT), C.POINTER(CurveT), ip, C.c_double, C.c_double, C.c_double,
                                   C.POINTER(OptionsT), C.POINTER(vp)]
        L.ccgmg_create_many.argtypes = [C.POINTER(ProblemT), ip, C.POINTER(OptionsT), ip, C.POINTER(vp)]
        L.ccgmg_query.argtypes = [vp, C.POINTER(InfoT)]
        L.ccgmg_get_cell_kinds.argtypes = [vp, ip, vp, vp]
        L.ccgmg_get_level_shape.argtypes = [vp, ip, C.POINTER(ip), C.POINTER(ip)]
        L.ccgmg_get_volumes.argtypes = [vp, ip, vp]
        L.ccgmg_get_counts.argtypes = [vp, ip, C.POINTER(C.c_long), C.POINTER(C.c_long)]
        L.ccgmg_get_irregular.argtypes = [vp, ip, vp, vp, vp, vp]
        L.ccgmg_get_stencils.argtypes = [vp, ip, vp, vp, vp]
        L.ccgmg_get_boundary_faces.argtypes = [vp, vp, vp, vp]
        L.ccgmg_get_alg3_order.argtypes = [vp, ip, vp]
        L.ccgmg_cell_quadrature.argtypes = [vp, C.POINTER(C.c_long), vp, vp, vp, vp]
        L.ccgmg_face_quadrature.argtypes = [vp, C.POINTER(C.c_long), vp, vp, vp, vp, vp, vp]
        L.ccgmg_apply.argtypes = [vp, vp, vp]
        L.ccgmg_residual_norms.argtypes = [vp, vp, vp, ip, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ccgmg_residual_norms_noalloc.argtypes = [vp, vp, vp, ip, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ccgmg_set_boundary.argtypes = [vp, vp, ip]
        L.ccgmg_solve.argtypes = [vp, vp, vp, ip, C.POINTER(ReportT)]
        L.ccgmg_solve_adjoint.argtypes = [vp, vp, vp, ip, C.POINTER(ReportT)]
        L.ccgmg_apply_adjoint.argtypes = [vp, vp, vp]
        L.ccgmg_apply_NT.argtypes = [vp, vp, vp, ip]
        L.ccgmg_profile_kernel.argtypes = [vp, ip, ip, ip, C.POINTER(C.c_double)]
        L.ccgmg_get_tuning.argtypes = [vp, ip, C.POINTER(ip), C.POINTER(ip)]
        L.ccgmg_get_smo2_stats.argtypes = [vp, ip, ip, C.POINTER(C.c_long)]
        L.ccgmg_tune.argtypes = [vp, vp]
        L.ccgmg_batch_create.argtypes = [C.POINTER(vp), ip, ip, C.POINTER(vp)]
        L.ccgmg_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(ip), C.POINTER(ReportT)]
        L.ccgmg_batch_last_error.argtypes = [vp]
        L.ccgmg_batch_last_error.restype = C.c_char_p
        L.ccgmg_batch_destroy.argtypes = [vp]
        L.ccgmg_batch_destroy.restype = None
        L.ccgmg_last_error.argtypes = [vp]
        L.ccgmg_last_error.restype = C.c_char_p
        L.ccgmg_create_error.argtypes = []
        L.ccgmg_create_error.restype = C.c_char_p
        L.ccgmg_destroy.argtypes = [vp]
        L.ccgmg_destroy.restype = None
        _LIB = L
    return _LIB


class CcgmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def default_options(**kw):
    o = OptionsT()
    lib().ccgmg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(a):
    """Raw pointer of a host numpy array (query results)."""
    if a is None:
        return None
    return a.ctypes.data


def _dev(t, n, name):
    """Raw pointer of a device array handed to the kernels: a torch GPU
    tensor of float64, contiguous, with exactly n elements.  Anything else
    is refused here, before the library sees the pointer."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor on the GPU, got %s" % (name, type(t).__name__))
    if not t.is_cuda:
        raise ValueError("%s must be on the GPU, got device %s" % (name, t.device))
    if t.dtype != torch.float64:
        raise ValueError("%s must be float64, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return t.data_ptr()


def _count(nrhs, name="nrhs"):
    if not isinstance(nrhs, (int, np.integer)) or nrhs < 1:
        raise ValueError("%s must be a positive integer, got %r" % (name, nrhs))
    return int(nrhs)


def _grid_t(grid):
    return GridT(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])


def _curves_t(curves):
    cs = (CurveT * len(curves))()
    for k, cu in enumerate(curves):
        cs[k].kind = cu["kind"]
        for t, v in enumerate(cu["p"]):
            cs[k].p[t] = v
        cs[k].domain_inside = cu["inside"]
        cs[k].bc = cu["bc"]
        for t, v in enumerate(cu.get("robin", (0.0, 0.0))):
            cs[k].robin[t] = v
    return cs


class Solver:
    """One context: geometry and coefficients fixed at construction."""

    def __init__(self, grid, curves, a, b, c, _ctx=None, _options=None, **options):
        L = lib()
        self.nx, self.ny = grid["nx"], grid["ny"]
        if _ctx is not None:   # made by create_many
            self.options, self.ctx = _options, _ctx
            self.info = self.query()
            return
        g = _grid_t(grid)
        cs = _curves_t(curves)
        self.options = default_options(**options)
        self.ctx = C.c_void_p()
        st = L.ccgmg_create(C.byref(g), cs, len(curves), a, b, c, C.byref(self.options), C.byref(self.ctx))
        if st != OK:
            raise CcgmgError(st, L.ccgmg_create_error().decode())
        self.info = self.query()

    def _check(self, st):
        if st != OK:
            raise CcgmgError(st, lib().ccgmg_last_error(self.ctx).decode())

    def close(self):
        if self.ctx:
            lib().ccgmg_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries -----------------------------------------------------------------
    def query(self):
        i = InfoT()
        self._check(lib().ccgmg_query(self.ctx, C.byref(i)))
        return {f: getattr(i, f) for f, _ in InfoT._fields_}

    def level_shape(self, level):
        nx, ny = C.c_int(), C.c_int()
        self._check(lib().ccgmg_get_level_shape(self.ctx, level, C.byref(nx), C.byref(ny)))
        return nx.value, ny.value

    def kinds(self, level=0):
        nx, ny = self.level_shape(level)
        k = np.zeros(nx * ny, dtype=np.int8)
        h = np.zeros(nx * ny, dtype=np.int32)
        self._check(lib().ccgmg_get_cell_kinds(self.ctx, level, _ptr(k), _ptr(h)))
        return k, h

    def volumes(self, level=0):
        nx, ny = self.level_shape(level)
        v = np.zeros(nx * ny)
        self._check(lib().ccgmg_get_volumes(self.ctx, level, _ptr(v)))
        return v

    def counts(self, level=0):
        ni, nf = C.c_long(), C.c_long()
        self._check(lib().ccgmg_get_counts(self.ctx, level, C.byref(ni), C.byref(nf)))
        return ni.value, nf.value

    def irregular(self, level=0):
        ni, _ = self.counts(level)
        rows = np.zeros(ni, dtype=np.int32)
        cols = np.zeros(ni * 15, dtype=np.int32)
        vals = np.zeros(ni * 15)
        cond = np.zeros(ni)
        self._check(lib().ccgmg_get_irregular(self.ctx, level, _ptr(rows), _ptr(cols), _ptr(vals), _ptr(cond)))
        return rows, cols.reshape(ni, 15), vals.reshape(ni, 15), cond

    def stencils(self, level=0):
        """(rows, cols, weights) of the least-squares rows (ccgmg_get_stencils)."""
        ni, _ = self.counts(level)
        rows = np.zeros(ni, dtype=np.int32)
        cols = np.zeros(ni * 15, dtype=np.int32)
        vals = np.zeros(ni * 15)
        self._check(lib().ccgmg_get_stencils(self.ctx, level, _ptr(rows), _ptr(cols), _ptr(vals)))
        return rows, cols.reshape(ni, 15), vals.reshape(ni, 15)

    def boundary_faces(self):
        nf = self.info["n_bdry_faces"]
        cell = np.zeros(nf, dtype=np.int32)
        curve = np.zeros(nf, dtype=np.int32)
        w = np.zeros(nf)
        self._check(lib().ccgmg_get_boundary_faces(self.ctx, _ptr(cell), _ptr(curve), _ptr(w)))
        return cell, curve, w

    def alg3_order(self, level=0):
        ni, _ = self.counts(level)
        p = np.zeros(ni, dtype=np.int32)
        self._check(lib().ccgmg_get_alg3_order(self.ctx, level, _ptr(p)))
        return p

    def cell_quadrature(self):
        n = C.c_long(0)
        self._check(lib().ccgmg_cell_quadrature(self.ctx, C.byref(n), None, None, None, None))
        cell = np.zeros(n.value, dtype=np.int32)
        x, y, w = np.zeros(n.value), np.zeros(n.value), np.zeros(n.value)
        self._check(lib().ccgmg_cell_quadrature(self.ctx, C.byref(n), _ptr(cell), _ptr(x), _ptr(y), _ptr(w)))
        return cell, x, y, w

    def face_quadrature(self):
        n = C.c_long(0)
        self._check(lib().ccgmg_face_quadrature(self.ctx, C.byref(n), None, None, None, None, None, None))
        out = [np.zeros(n.value, dtype=np.int32)] + [np.zeros(n.value) for _ in range(5)]
        self._check(lib().ccgmg_face_quadrature(self.ctx, C.byref(n), *[_ptr(a) for a in out]))
        return tuple(out)

    # -- device calls ------------------------------------------------------------
    @property
    def n_cells(self):
        return self.nx * self.ny

    def apply(self, u, out):
        n = self.n_cells
        self._check(lib().ccgmg_apply(self.ctx, _dev(u, n, "u"), _dev(out, n, "out")))

    def residual_norms(self, f, u, nrhs=1):
        """Relative L-infinity and L2 residual norms of the iterate u (one
        value per right-hand side), with the boundary data last set."""
        nrhs = _count(nrhs)
        n = nrhs * self.n_cells
        ri, r2 = (C.c_double * nrhs)(), (C.c_double * nrhs)()
        self._check(lib().ccgmg_residual_norms(self.ctx, _dev(f, n, "f"), _dev(u, n, "u"), nrhs, ri, r2))
        return list(ri), list(r2)

    def residual_norms_noalloc(self, f, u, nrhs=1):
        """residual_norms through ccgmg_residual_norms_noalloc (the library's
        static device scratch; no allocation in the library)."""
        nrhs = _count(nrhs)
        n = nrhs * self.n_cells
        ri, r2 = (C.c_double * nrhs)(), (C.c_double * nrhs)()
        self._check(lib().ccgmg_residual_norms_noalloc(self.ctx, _dev(f, n, "f"), _dev(u, n, "u"), nrhs, ri, r2))
        return list(ri), list(r2)

    def set_boundary(self, g, nrhs=1):
        """Boundary data for nrhs right-hand sides ([nrhs][n_bdry_faces]);
        nrhs = 0 drops the boundary term."""
        if nrhs == 0:
            self._check(lib().ccgmg_set_boundary(self.ctx, None, 0))
            return
        nrhs = _count(nrhs)
        nf = self.info["n_bdry_faces"]
        ptr = _dev(g, nrhs * nf, "g") if nf > 0 else None
        self._check(lib().ccgmg_set_boundary(self.ctx, ptr, nrhs))

    def solve(self, f, u, nrhs=1, raise_on_noconv=True):
        nrhs = _count(nrhs)
        n = nrhs * self.n_cells
        rep = ReportT()
        st = lib().ccgmg_solve(self.ctx, _dev(f, n, "f"), _dev(u, n, "u"), nrhs, C.byref(rep))
        if st != OK and (raise_on_noconv or st != ENOCONV):
            self._check(st)
        return _report(rep, st)

    def solve_adjoint(self, rhs, lam, nrhs=1, raise_on_noconv=True):
        nrhs = _count(nrhs)
        n = nrhs * self.n_cells
        rep = ReportT()
        st = lib().ccgmg_solve_adjoint(self.ctx, _dev(rhs, n, "rhs"), _dev(lam, n, "lam"), nrhs, C.byref(rep))
        if st != OK and (raise_on_noconv or st != ENOCONV):
            self._check(st)
        return _report(rep, st)

    def tune(self, f):
        """Re-choose schedule, depth and (with tune_schedule) the SMO-1
        weight by timing solves of this right-hand side (with the boundary
        data last set); refreshes ``info``."""
        self._check(lib().ccgmg_tune(self.ctx, _dev(f, self.n_cells, "f")))
        self.info = self.query()

    def profile_kernel(self, kernel, level=0, reps=50):
        """Mean duration (microseconds) of one V-cycle kernel, HIP events."""
        us = C.c_double()
        self._check(lib().ccgmg_profile_kernel(self.ctx, kernel, level, reps, C.byref(us)))
        return us.value

    def tuning(self, level=0):
        """SMO-1 tile heights (FP64, FP32) picked for a level at set-up."""
        a, b = C.c_int(), C.c_int()
        self._check(lib().ccgmg_get_tuning(self.ctx, level, C.byref(a), C.byref(b)))
        return a.value, b.value

    def smo2_stats(self, level=0, adjoint=False):
        """SMO-2 block data sizes: blocks, block rows, overlapped rows, their
        CSR entries, inverse bytes."""
        st = (C.c_long * 5)()
        self._check(lib().ccgmg_get_smo2_stats(self.ctx, level, int(adjoint), st))
        keys = ("blocks", "rows", "ext_rows", "ext_nnz", "inv_bytes")
        return dict(zip(keys, list(st)))

    def apply_adjoint(self, lam, out):
        n = self.n_cells
        self._check(lib().ccgmg_apply_adjoint(self.ctx, _dev(lam, n, "lam"), _dev(out, n, "out")))

    def apply_NT(self, lam, out, nrhs=1):
        nrhs = _count(nrhs)
        nf = self.info["n_bdry_faces"]
        self._check(lib().ccgmg_apply_NT(self.ctx, _dev(lam, nrhs * self.n_cells, "lam"),
                                         _dev(out, nrhs * nf, "out"), nrhs))


def create_many(problems, options=None, host_threads=0):
    """Solvers for several geometries, set up together (ccgmg_create_many):
    problems is a list of (grid, curves, a, b, c); options a list of option
    dicts (one per problem) or None."""
    L = lib()
    n = len(problems)
    if n < 1:
        raise ValueError("no problems")
    opts = options or [{}] * n
    if len(opts) != n:
        raise ValueError("one options dict per problem")
    keep = []
    P = (ProblemT * n)()
    O = (OptionsT * n)()
    for k, ((grid, curves, a, b, c), o) in enumerate(zip(problems, opts)):
        cs = _curves_t(curves)
        keep.append(cs)
        P[k].grid = _grid_t(grid)
        P[k].curves = C.cast(cs, C.POINTER(CurveT))
        P[k].ncurves = len(curves)
        P[k].a, P[k].b, P[k].c = a, b, c
        O[k] = default_options(**o)
    out = (C.c_void_p * n)()
    st = L.ccgmg_create_many(P, n, O, int(host_threads), out)
    if st != OK:
        raise CcgmgError(st, L.ccgmg_create_error().decode())
    return [Solver(p[0], p[1], p[2], p[3], p[4], _ctx=C.c_void_p(out[k]), _options=O[k])
            for k, p in enumerate(problems)]


def _report(rep, st):
    return {"status": st, "cycles": rep.cycles, "outer_iters": rep.outer_iters, "rel_res_inf": rep.rel_res_inf,
            "rel_res_2": rep.rel_res_2,
            "seconds": rep.seconds, "history": list(rep.history[:min(64, max(rep.cycles, 0))])}


class Batch:
    """Several Solver contexts (different geometries) solved together: one
    captured V-cycle of every geometry per graph replay (ccgmg_batch_*)."""

    def __init__(self, solvers, nbranches=4):
        L = lib()
        self.solvers = list(solvers)      # keeps the contexts alive
        arr = (C.c_void_p * len(self.solvers))(*[S.ctx.value for S in self.solvers])
        self.h = C.c_void_p()
        st = L.ccgmg_batch_create(arr, len(self.solvers), nbranches, C.byref(self.h))
        if st != OK:
            raise CcgmgError(st, L.ccgmg_create_error().decode())

    def solve(self, fs, us, nrhs=None, raise_on_noconv=True):
        n = len(self.solvers)
        if len(fs) != n or len(us) != n:
            raise ValueError("one right-hand side and one solution array per geometry")
        nr = [_count(v) for v in (nrhs or [1] * n)]
        if len(nr) != n:
            raise ValueError("one right-hand-side count per geometry")
        fa = (C.c_void_p * n)(*[_dev(f, m * S.n_cells, "f[%d]" % k)
                                for k, (f, m, S) in enumerate(zip(fs, nr, self.solvers))])
        ua = (C.c_void_p * n)(*[_dev(u, m * S.n_cells, "u[%d]" % k)
                                for k, (u, m, S) in enumerate(zip(us, nr, self.solvers))])
        na = (C.c_int * n)(*nr)
        reps = (ReportT * n)()
        st = lib().ccgmg_batch_solve(self.h, fa, ua, na, reps)
        if st != OK and (raise_on_noconv or st != ENOCONV):
            raise CcgmgError(st, lib().ccgmg_batch_last_error(self.h).decode())
        return [_report(r, st) for r in reps]

    def close(self):
        if self.h:
            lib().ccgmg_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
