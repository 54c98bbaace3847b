"""Pins of the oracle's solution and multigrid (Sections 3.4, 4, 5)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle.discretization import boundary_data
from oracle.geometry import cell_averages
from oracle.multigrid import (Hierarchy, Level, alg3_order, cyclic_bandwidth, direct_solve,
                              direct_solve_transpose, rhs_vector)
from oracle.norms import norms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _errors(cfg, n):
    lv = Level(cfg["grid"] if n is None else W.grid(n), cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
    sol = cfg["solution"]
    f = cell_averages(lv.cg, cfg["f"])
    g = boundary_data(lv.disc, sol)
    u = direct_solve(lv, rhs_vector(lv, f, g))
    ue = cell_averages(lv.cg, sol.u).ravel()
    return norms(u - ue, lv.cg.vol), lv, u, f, g


def test_problem2_dirichlet_matches_paper_table():
    """Problem 2 with Dirichlet data on the ellipse (Table tab:errorsOfEllipseDD):
    same magnitude as the paper at h = 1/64, 1/128 and a fourth-order rate."""
    gold = json.load(open(os.path.join(GOLDEN, "problem2_errors.json")))["dirichlet_ellipse"]
    errs = []
    for k, n in enumerate((64, 128)):
        (l1, l2, li), *_ = _errors(W.problem2(n, hole_bc=W.DIRICHLET), None)
        errs.append((l1, l2, li))
        for got, ref in zip((li, l1, l2), (gold["Linf"][k], gold["L1"][k], gold["L2"][k])):
            assert ref / 5 < got < ref * 5, (n, got, ref)
    rates = np.log2(np.array(errs[0]) / np.array(errs[1]))
    assert np.all(rates > 3.5) and np.all(rates < 5.5), rates


def test_problem2_neumann_fourth_order():
    gold = json.load(open(os.path.join(GOLDEN, "problem2_errors.json")))["neumann_ellipse"]
    (l1a, l2a, lia), *_ = _errors(W.problem2(64, hole_bc=W.NEUMANN), None)
    (l1b, l2b, lib), *_ = _errors(W.problem2(128, hole_bc=W.NEUMANN), None)
    assert gold["Linf"][1] / 10 < lib < gold["Linf"][1] * 10
    for a, b in ((l1a, l1b), (l2a, l2b), (lia, lib)):
        assert 3.5 < np.log2(a / b) < 5.0


@pytest.mark.slow
def test_smallest_condition_lattice_pick_measured():
    """The measured alternative to R-PLG's lattice pick (the paper gives no
    algorithm, Section 2.2): keeping the acceptable lattice with the smallest
    condition number instead of the smallest W^-1-norm.  On Problem 2 with
    Neumann data on the ellipse (Table tab:errorsOfEllipseDN) its L-infinity
    error at h = 1/128 is within 2x of the paper's and below the min-norm
    pick's (3.6x the paper's there), but on the five-ellipse b = 1.2 workload
    at 128^2 the oracle's two-level V-cycle with it does not converge (the
    residual grows), which the min-norm pick avoids: the library keeps the
    latter.  The divergence is grid-specific (the same workload at 64^2 and
    96^2 converges with either pick); the test pins the grid where it shows."""
    import oracle_jobs
    gold = json.load(open(os.path.join(GOLDEN, "problem2_errors.json")))["neumann_ellipse"]
    rules = ("min_norm", "min_cond")
    with oracle_jobs.pool(4) as ex:
        errs = ex.map(oracle_jobs.lattice_rule_p2n_error, rules, [128] * 2)
        hists = ex.map(oracle_jobs.lattice_rule_vcycle_history, rules, [5] * 2, [128] * 2, [8] * 2)
        li = dict(zip(rules, errs))
        hist = dict(zip(rules, hists))
    print("P2N h=1/128 Linf: min-norm %.3e, min-cond %.3e, paper %.3e" % (li["min_norm"], li["min_cond"],
                                                                        gold["Linf"][1]))
    assert li["min_cond"] < li["min_norm"]
    assert gold["Linf"][1] / 2 < li["min_cond"] < 2 * gold["Linf"][1]
    assert li["min_norm"] > 2 * gold["Linf"][1]
    print("five ellipses 128^2, 2 levels: min-norm %s, min-cond %s" % (
        " ".join("%.1e" % v for v in hist["min_norm"][-3:]), " ".join("%.1e" % v for v in hist["min_cond"][-3:])))
    assert hist["min_norm"][-1] < hist["min_norm"][0]
    assert not (hist["min_cond"][-1] < hist["min_cond"][0])


def test_exact_recovery_of_quartic():
    """u in Pi_4 is reproduced to rounding (the discretization is exact on Pi_4)."""
    cfg = W.config(2, n=32)
    sol = W.polynomial({(4, 0): 1.0, (2, 2): -0.5, (1, 1): 2.0, (0, 3): 0.25, (0, 0): 1.0})
    cfg = dict(cfg, solution=sol, f=sol.f(cfg["a"], cfg["b"], cfg["c"]))
    (l1, l2, li), *_ = _errors(cfg, None)
    assert li < 1e-11


def test_dense_brute_force_and_gmg_agree():
    cfg = W.config(1, n=16)
    lv = Level(W.grid(16), cfg["curves"], 1.0, 0.0, 1.0)
    r = np.random.default_rng(3).standard_normal(16 * 16) * lv.nonempty
    ne = lv.ne_idx
    dense = np.linalg.solve(lv.L[ne][:, ne].toarray(), r[ne])
    sparse = direct_solve(lv, r)[ne]
    assert np.max(np.abs(dense - sparse)) < 1e-12 * np.max(np.abs(dense))
    cfg = W.config(1, n=32)
    H = Hierarchy(cfg["grid"], cfg["curves"], 1.0, 0.0, 1.0)
    H.select_depth()
    lv = H.levels[0]
    r = np.random.default_rng(4).standard_normal(32 * 32) * lv.nonempty
    hist = []
    u = H.solve(r, tol=1e-13, history=hist)
    ud = direct_solve(lv, r)
    assert np.max(np.abs(u - ud)) < 1e-11 * np.max(np.abs(ud))
    assert all(b < a for a, b in zip(hist, hist[1:]))          # monotone decrease


def test_smo2_zeroes_irregular_residual():
    """After SMO-2 the residual of the irregular rows vanishes (Section 4.1)."""
    cfg = W.config(4, n=64)
    H = Hierarchy(cfg["grid"], cfg["curves"], 1.0, 0.0, 1.0, max_levels=2)
    lv = H.levels[0]
    r = np.random.default_rng(5).standard_normal(lv.nx * lv.ny) * lv.nonempty
    u = H.smooth(0, np.zeros_like(r), r, 0.5)
    res = r - lv.L @ u
    assert np.max(np.abs(res[lv.irr])) < 1e-12 * np.max(np.abs(r))
    assert np.max(np.abs(res[lv.reg])) > 1e-3


def test_transpose_solve():
    cfg = W.config(2, n=32)
    lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
    rng = np.random.default_rng(6)
    r = rng.standard_normal(lv.nx * lv.ny) * lv.nonempty
    lam = direct_solve_transpose(lv, r)
    ne = lv.ne_idx
    assert np.max(np.abs(lv.L[ne][:, ne].T @ lam[ne] - r[ne])) < 1e-9 * np.max(np.abs(r))
    u = rng.standard_normal(lv.nx * lv.ny) * lv.nonempty
    v = rng.standard_normal(lv.nx * lv.ny) * lv.nonempty
    lhs = np.dot(lv.L @ u, v)
    rhs = np.dot(u, lv.L.T @ v)
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(lv.L @ u) * np.linalg.norm(v)


def test_alg3_order_is_permutation_with_bounded_bandwidth():
    bws = []
    for n in (64, 128):
        lv = Level(W.grid(n), [W.box(), W.circle(0.5, 0.5, 0.2)], 1.0, 0.0, 1.0)
        order = alg3_order(lv.disc)
        assert np.array_equal(np.sort(order), np.arange(lv.irr.size))
        bws.append(cyclic_bandwidth(lv))
    # independent of h and small (Section 4.2 reports <= 20 for its own numbering)
    assert max(bws) <= 32 and bws[1] <= bws[0] + 2


def test_norms_normalisation():
    vol = np.array([0.0, 1.0, 0.5, 0.25])
    assert norms(np.full(4, -3.0), vol) == (3.0, 3.0, 3.0)


def test_problem1_matches_paper_tables():
    """Problem 1 (Section 5.1; Tables tab:truncationErrorsOfProblem1 and
    tab:solutionErrorsOfProblem1): truncation and solution errors at
    h = 1/40 and 1/80 of the paper's magnitude, fourth-order solution error
    and about fourth-order L1 truncation error.  The flower is tangent to the
    grid lines y = +-0.2 at x = 0, which exercises the tangency reading of
    the cut-cell construction."""
    from oracle.norms import norms as _norms
    gold = json.load(open(os.path.join(GOLDEN, "problem1_errors.json")))
    tau, err = [], []
    for n in (40, 80):
        cfg = W.problem1(n)
        lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
        f = cell_averages(lv.cg, cfg["f"]).ravel()
        g = boundary_data(lv.disc, cfg["solution"])
        ue = cell_averages(lv.cg, cfg["solution"].u).ravel()
        N = lv.disc.matrices()[1]
        tau.append(_norms((lv.L @ ue + N @ g - f) * lv.nonempty, lv.cg.vol))
        u = direct_solve(lv, rhs_vector(lv, f, g))
        err.append(_norms((u - ue) * lv.nonempty, lv.cg.vol))
    for k in range(2):
        for key, idx in (("L1", 0), ("L2", 1), ("Linf", 2)):
            for got, table in ((tau[k][idx], gold["truncation"][key][k]), (err[k][idx], gold["solution"][key][k])):
                assert table / 5 < got < table * 5, (k, key, got, table)
    sol_rates = np.log2(np.array(err[0]) / np.array(err[1]))
    assert np.all(sol_rates > 3.3) and np.all(sol_rates < 5.5), sol_rates
    assert np.log2(tau[0][0] / tau[1][0]) > 3.0


def test_problem3_matches_paper_table():
    """Problem 3 case (i) (Section 5.1, Table tab:errorsOfBox): (a,b,c) =
    (1,0,2) on the unit box, u = sin(4x) cos(3y); oracle direct solutions
    against the exact cell averages at h = 1/64 and 1/128 within 30% of the
    table in every norm, and fourth order."""
    from oracle.norms import norms as _norms
    p3 = json.load(open(os.path.join(GOLDEN, "problem3_errors.json")))
    e3 = []
    for n in (64, 128):
        cfg = W.problem3(n)
        lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
        f = cell_averages(lv.cg, cfg["f"]).ravel()
        g = boundary_data(lv.disc, cfg["solution"])
        ue = cell_averages(lv.cg, cfg["solution"].u).ravel()
        u = direct_solve(lv, rhs_vector(lv, f, g))
        e3.append(dict(zip(("L1", "L2", "Linf"), _norms((u - ue) * lv.nonempty, lv.cg.vol))))
    for k in range(2):
        for norm in ("L1", "L2", "Linf"):
            table = p3["case_i"][norm][k]
            assert table / 1.3 < e3[k][norm] < table * 1.3, (k, norm, e3[k][norm], table)
    for norm in ("L1", "L2", "Linf"):
        assert 3.7 < np.log2(e3[0][norm] / e3[1][norm]) < 4.5


def test_problem2_robin_fourth_order():
    """Problem 2's domain and solution with the Robin condition u + 0.5 du/dn
    = g on the ellipse (the boundary operator of Section 3; the paper has no
    Robin table, so the magnitude is parity unpinned): oracle direct solutions
    at h = 1/64 and 1/128 converge at fourth order in every norm, with errors
    between those of the Dirichlet and Neumann variants at h = 1/64."""
    from oracle.norms import norms as _norms

    def errors(name, n):
        cfg = W.problem(name, n)
        lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
        f = cell_averages(lv.cg, cfg["f"]).ravel()
        g = boundary_data(lv.disc, cfg["solution"])
        ue = cell_averages(lv.cg, cfg["solution"].u).ravel()
        u = direct_solve(lv, rhs_vector(lv, f, g))
        return np.array(_norms((u - ue) * lv.nonempty, lv.cg.vol))

    ea, eb = errors("P2R", 64), errors("P2R", 128)
    rates = np.log2(ea / eb)
    assert np.all(rates > 3.5) and np.all(rates < 5.0), rates
    gold = json.load(open(os.path.join(GOLDEN, "problem2_errors.json")))
    assert gold["dirichlet_ellipse"]["Linf"][0] / 5 < ea[2] < gold["neumann_ellipse"]["Linf"][0] * 10


def test_problem3_rotated_box_matches_paper_table():
    """Problem 3 case (ii) (Section 5.1, Table tab:errorsOfBox): the unit box
    rotated by pi/6 (a polygon curve; corner cells of the cut-cell grid),
    (a,b,c) = (5/4, -sqrt(3)/2, 7/4); oracle direct solutions at h = 1/64 and
    1/128 within a factor 3 of the table in every norm (measured 1.4-2.1),
    and fourth order."""
    from oracle.norms import norms as _norms
    p3 = json.load(open(os.path.join(GOLDEN, "problem3_errors.json")))
    e = []
    for n in (64, 128):
        cfg = W.problem3_rotated(n)
        lv = Level(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
        f = cell_averages(lv.cg, cfg["f"]).ravel()
        g = boundary_data(lv.disc, cfg["solution"])
        ue = cell_averages(lv.cg, cfg["solution"].u).ravel()
        u = direct_solve(lv, rhs_vector(lv, f, g))
        e.append(dict(zip(("L1", "L2", "Linf"), _norms((u - ue) * lv.nonempty, lv.cg.vol))))
    for k in range(2):
        for norm in ("L1", "L2", "Linf"):
            table = p3["case_ii"][norm][k]
            assert table / 3 < e[k][norm] < table * 3, (k, norm, e[k][norm], table)
    for norm in ("L1", "L2", "Linf"):
        assert 3.7 < np.log2(e[0][norm] / e[1][norm]) < 5.0


def _problem2_hierarchy(n, bc="P2D"):
    cfg = W.problem(bc, n)
    H = Hierarchy(cfg["grid"], cfg["curves"], cfg["a"], cfg["b"], cfg["c"])
    lv = H.levels[0]
    f = cell_averages(lv.cg, cfg["f"]).ravel()
    g = boundary_data(lv.disc, cfg["solution"])
    return H, rhs_vector(lv, f, g)


def test_fmg_with_one_level_is_the_direct_solve():
    """With the hierarchy cut to the finest level, an FMG cycle is the
    bottom solver alone: the exact solution in one iteration."""
    H, r = _problem2_hierarchy(32)
    while H.M > 0:
        H.levels.pop()
    H._factor_bottom()
    ref = direct_solve(H.levels[0], r)
    e = H.fmg_cycle(r)
    assert np.max(np.abs(e - ref)) <= 1e-13 * np.max(np.abs(ref))
    hist = []
    H.solve_fmg(r, tol=1e-12, history=hist)
    assert len(hist) == 1 and hist[0] <= 1e-12


def test_fmg_cycle_is_linear_and_converges_to_the_direct_solve():
    """An FMG cycle from a zero guess is a linear map of its right-hand side
    (restriction, LU, prolongation and smoothing are linear), and FMG
    iterations converge to the direct solution of L u = f - N g."""
    H, r = _problem2_hierarchy(64)
    assert H.M >= 2
    rng = np.random.default_rng(5)
    r2 = rng.standard_normal(r.size) * H.levels[0].nonempty
    a, b = 0.7, -1.9
    lhs = H.fmg_cycle(a * r + b * r2)
    rhs = a * H.fmg_cycle(r) + b * H.fmg_cycle(r2)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
    u = H.solve_fmg(r, tol=1e-12)
    ref = direct_solve(H.levels[0], r)
    assert np.max(np.abs(u - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_fmg_residual_reduction_of_the_order_of_the_paper():
    """Section 5.2, Fig. fig:reduction: on Problem 2 at h = 1/128 with
    omega = 0.5, nu1 = nu2 = 3 and a zero initial guess, the relative
    residual falls by a factor of 11.3 per FMG cycle iteration.  The
    oracle's FMG (the descent by Alg. 2's restriction, the bottom solve, and
    one V-cycle per level on the way up from the prolonged coarser
    solution) must reduce it by a factor within x2 of that, and by more per
    iteration than a V-cycle does."""
    H, r = _problem2_hierarchy(128)
    hf, hv = [], []
    H.solve_fmg(r, tol=0.0, max_cycles=8, history=hf)
    H.solve(r, tol=0.0, max_cycles=8, history=hv)
    assert len(hf) == 8 and len(hv) == 8          # no stagnation or divergence on the way
    fmg = (hf[0] / hf[7]) ** (1.0 / 7)
    vc = (hv[0] / hv[7]) ** (1.0 / 7)
    print("residual reduction per iteration: FMG %.1f, V-cycle %.1f (paper's FMG: 11.3)" % (fmg, vc))
    assert 11.3 / 2 <= fmg <= 11.3 * 2
    assert fmg > vc
