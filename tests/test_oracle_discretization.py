"""Pins of the oracle's discretization (Sections 2.2-2.3, 3.2-3.4)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle.discretization import (BASIS, D4, T0, _CANDIDATES, _LINE_ASSIGN, Discretization,
                                   boundary_data, regular_coefficients)
from oracle.geometry import build_cut_grid, cell_averages


def _square_avg(a, d):
    """Exact average of X^a over the unit interval centred at d (rational)."""
    d = Fraction(d)
    return ((d + Fraction(1, 2)) ** (a + 1) - (d - Fraction(1, 2)) ** (a + 1)) / (a + 1)


def test_regular_stencil_exact_to_degree_five():
    """eq. stdLap / stdGrad: applied to exact cell averages of x^p y^q
    (p+q <= 5, h = 1) the regular rows return the exact average of
    a u_xx + b u_xy + c u_yy."""
    a, b, c = Fraction(3, 2), Fraction(1, 3), Fraction(2)
    co = regular_coefficients(1.5, 1.0 / 3.0, 2.0, 1.0)
    g = {1: 8, 2: -1, -1: -8, -2: 1}
    for p in range(6):
        for q in range(6 - p):
            # regular stencil with exact coefficients
            lhs = Fraction(0)
            for (dx, dy) in co:
                if dx == 0 and dy == 0:
                    w = -30 * (a + c) / 12
                elif dy == 0:
                    w = a * (16 if abs(dx) == 1 else -1) / 12
                elif dx == 0:
                    w = c * (16 if abs(dy) == 1 else -1) / 12
                else:
                    w = b * g[dx] * g[dy] / 144
                assert abs(float(w) - co[(dx, dy)]) < 1e-15 * max(1.0, abs(float(w)))
                lhs += w * _square_avg(p, dx) * _square_avg(q, dy)
            rhs = Fraction(0)
            if p >= 2:
                rhs += a * p * (p - 1) * _square_avg(p - 2, 0) * _square_avg(q, 0)
            if p >= 1 and q >= 1:
                rhs += b * p * q * _square_avg(p - 1, 0) * _square_avg(q - 1, 0)
            if q >= 2:
                rhs += c * q * (q - 1) * _square_avg(p, 0) * _square_avg(q - 2, 0)
            assert lhs == rhs, (p, q)
    assert abs(sum(co.values())) < 1e-12


def _det_fraction(M):
    M = [[Fraction(v) for v in row] for row in M]
    n = len(M)
    det = Fraction(1)
    for k in range(n):
        piv = next((r for r in range(k, n) if M[r][k] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != k:
            M[k], M[piv] = M[piv], M[k]
            det = -det
        det *= M[k][k]
        for r in range(k + 1, n):
            f = M[r][k] / M[k][k]
            for col in range(k, n):
                M[r][col] -= f * M[k][col]
    return det


def test_lattice_families_poised():
    """Every principal-lattice image and every line-lattice shape is poised
    for degree-4 point interpolation: the integer Vandermonde matrix has a
    non-zero exact determinant (Definition of poisedness, eq. sampleMatrix)."""
    for offs in _CANDIDATES[:20] + _CANDIDATES[-5:]:
        V = [[x ** a * y ** b for (a, b) in BASIS] for (x, y) in offs]
        assert _det_fraction(V) != 0
    rng = np.random.default_rng(0)
    for e in rng.choice(len(_LINE_ASSIGN), 12, replace=False):
        lines, counts = _LINE_ASSIGN[e]
        pts = []
        for d, k in zip(lines, counts):
            xs = rng.choice(np.arange(-4, 5), size=k, replace=False)
            pts += [(int(x), int(d)) for x in xs]
        V = [[x ** a * y ** b for (a, b) in BASIS] for (x, y) in pts]
        assert _det_fraction(V) != 0
    assert len(T0) == 15 and len(D4) == 8


def test_square_system_weights_are_exact_rationals():
    """Box-only domain: the cells of row 1 are irregular, own no boundary
    face, and their lattices hold pure cells only, so the weights solve a
    square rational system exactly.  The FP64 weights must match it."""
    n = 16
    cg = build_cut_grid(W.grid(n), [W.box()])
    a, b, c = 1.0, 0.5, 1.25
    d = Discretization(cg, a, b, c)
    A, B, C = Fraction(1), Fraction(1, 2), Fraction(5, 4)
    checked = 0
    for q in [1 * n + 5, 1 * n + 8, 8 * n + 1]:
        cells = d.stencils[q]
        assert not cg.faces(q)
        ii = [k % n for k in cells]
        jj = [k // n for k in cells]
        px = Fraction(min(ii) + max(ii) + 1, 2)
        py = Fraction(min(jj) + max(jj) + 1, 2)
        M = [[_square_avg(al, Fraction(k % n) + Fraction(1, 2) - px) *
              _square_avg(be, Fraction(k // n) + Fraction(1, 2) - py) for k in cells] for (al, be) in BASIS]
        dq = (Fraction(q % n) + Fraction(1, 2) - px, Fraction(q // n) + Fraction(1, 2) - py)
        L = []
        for al, be in BASIS:
            v = Fraction(0)
            if al >= 2:
                v += A * al * (al - 1) * _square_avg(al - 2, dq[0]) * _square_avg(be, dq[1])
            if al >= 1 and be >= 1:
                v += B * al * be * _square_avg(al - 1, dq[0]) * _square_avg(be - 1, dq[1])
            if be >= 2:
                v += C * be * (be - 1) * _square_avg(al, dq[0]) * _square_avg(be - 2, dq[1])
            L.append(v)
        # exact Gaussian elimination
        m = len(M)
        aug = [row[:] + [L[r]] for r, row in enumerate(M)]
        for k in range(m):
            piv = next(r for r in range(k, m) if aug[r][k] != 0)
            aug[k], aug[piv] = aug[piv], aug[k]
            for r in range(m):
                if r != k and aug[r][k] != 0:
                    f = aug[r][k] / aug[k][k]
                    aug[r] = [x - f * y for x, y in zip(aug[r], aug[k])]
        beta = [float(aug[r][m] / aug[r][r]) for r in range(m)]
        got = d.weights[q] * d.h * d.h
        cond = d.conds[q]
        assert np.max(np.abs(got - np.array(beta))) <= 50 * cond * 2.2e-16 * max(1.0, max(map(abs, beta)))
        checked += 1
    assert checked == 3


@pytest.mark.parametrize("k,n", [(1, 32), (2, 32), (4, 64), (5, 64)])
def test_plg_invariants_and_ls_exactness(k, n):
    cfg = W.config(k, n=n)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    d = Discretization(cg, cfg["a"], cfg["b"], cfg["c"])
    nx = d.nx
    for q in d.irregular[:: max(1, len(d.irregular) // 60)]:
        q = int(q)
        cells = d.stencils[q]
        assert len(set(cells)) == 15 and q in cells
        for j in cells:
            assert d.nonempty[j]
            assert max(abs(j % nx - q % nx), abs(j // nx - q // nx)) <= 4
        assert d.conds[q] <= 1e8
        assert d.weights[q][cells.index(q)] * d.h ** 2 <= -0.5 * (cfg["a"] + cfg["c"])
        # M beta = L-hat in scaled units and the KKT condition beta in range(W M^T)
        cond, beta, fkeys, w = d.fit(q, cells)
        p = d._bbox_centre(cells)
        cols = [d.basis_averages(j, p) for j in cells] + [d.face_column(q, cg.faces(q)[f], p) for f in fkeys]
        M = np.array(cols).T
        Lh = d.operator_averages(q, p)
        assert np.max(np.abs(M @ beta - Lh)) < 1e-12 * max(1.0, np.max(np.abs(Lh)))
        lam, *_ = np.linalg.lstsq((M / w).T, beta, rcond=None)
        assert np.max(np.abs((M / w).T @ lam - beta)) < 1e-10 * np.max(np.abs(beta))


@pytest.mark.parametrize("k,n", [(1, 32), (2, 64), (4, 64), (5, 32)])
def test_operator_exact_on_quartics(k, n):
    """L <u> + N <<Nu>> = <L u> on every non-empty cell for u in Pi_4
    (the design equation of the weights, Section 3.3)."""
    cfg = W.config(k, n=n)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    d = Discretization(cg, cfg["a"], cfg["b"], cfg["c"])
    rng = np.random.default_rng(k)
    sol = W.polynomial({(p, q): rng.standard_normal() for p in range(5) for q in range(5 - p)})
    u = cell_averages(cg, sol.u)
    f = cell_averages(cg, sol.f(cfg["a"], cfg["b"], cfg["c"]))
    g = boundary_data(d, sol)
    Lu = d.apply(u, g)
    ne = d.nonempty.reshape(d.ny, d.nx)
    scale = np.max(np.abs(u[ne])) / d.h ** 2
    assert np.max(np.abs(Lu - f)[ne]) < 1e-12 * scale


def test_regular_rows_exact_on_quintic():
    cfg = W.config(4, n=64)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    d = Discretization(cg, 1.0, 0.7, 1.3)
    sol = W.polynomial({(5, 0): 1.0, (3, 2): -2.0, (1, 4): 0.5, (0, 5): 1.5})
    u = cell_averages(cg, sol.u)
    f = cell_averages(cg, sol.f(1.0, 0.7, 1.3))
    Lu = d.apply(u)
    reg = d.regular.reshape(d.ny, d.nx)
    assert np.max(np.abs(Lu - f)[reg]) < 1e-12 * np.max(np.abs(u)) / d.h ** 2
    irr = (d.nonempty & ~d.regular).reshape(d.ny, d.nx)
    assert np.max(np.abs(Lu - f)[irr]) > 1e-9       # PLG rows are only degree-4 exact


def test_box_domain_kinds():
    n = 24
    cg = build_cut_grid(W.grid(n), [W.box()])
    d = Discretization(cg, 1.0, 0.0, 1.0)
    assert int(d.regular.sum()) == (n - 4) ** 2
    assert len(d.faces) == 4 * n - 4


@pytest.mark.parametrize("k,which,gammas", [(2, 1, (1.0, 0.5)), (1, 0, (0.7, 1.0)), (4, 0, (-0.3, 2.0))])
def test_operator_exact_on_quartics_with_robin_data(k, which, gammas):
    """L <u> + N <<(gamma1 + gamma2 d/dn) u>> = <L u> on every non-empty cell
    for u in Pi_4 with Robin data (the boundary operator of Section 3) on one
    curve: a hole with b != 0, an outer circle, and the box.  A wrong unit of
    the gradient part (h or 1/h), a wrong weight scaling or a flipped normal
    breaks the identity."""
    cfg = W.config(k, n=64)
    curves = list(cfg["curves"])
    curves[which] = W.robin(curves[which], *gammas)
    cg = build_cut_grid(cfg["grid"], curves)
    d = Discretization(cg, cfg["a"], cfg["b"], cfg["c"])
    rng = np.random.default_rng(30 + k)
    sol = W.polynomial({(p, q): rng.standard_normal() for p in range(5) for q in range(5 - p)})
    u = cell_averages(cg, sol.u)
    f = cell_averages(cg, sol.f(cfg["a"], cfg["b"], cfg["c"]))
    g = boundary_data(d, sol)
    Lu = d.apply(u, g)
    ne = d.nonempty.reshape(d.ny, d.nx)
    scale = np.max(np.abs(u[ne])) / d.h ** 2
    assert np.max(np.abs(Lu - f)[ne]) < 1e-12 * scale
    # the Robin faces carry weights (the rows do depend on the Robin data)
    robin_faces = [i for i, (_, c) in enumerate(d.faces) if c == which]
    assert robin_faces


def _brute_force_pool(disc, q, pool_size=16, radius=4):
    """The R-PLG pool by direct enumeration of the rule (module docstring of
    oracle.discretization): every image of the principal lattice and every
    line lattice, built cell by cell, kept if inside K, ranked by (sum of
    squared distances, largest infinity distance, family/axis, enumeration
    index), duplicates dropped, the first pool_size taken."""
    import itertools
    nx, ny = disc.nx, disc.ny
    qi, qj = q % nx, q // nx

    def feasible(dx, dy):
        i, j = qi + dx, qj + dy
        return 0 <= i < nx and 0 <= j < ny and bool(disc.nonempty[j * nx + i])

    def key_of(offs):
        return (sum(dx * dx + dy * dy for dx, dy in offs), max(max(abs(dx), abs(dy)) for dx, dy in offs))

    ranked = []
    # (a) q + g(T0 - t): symmetries id, rot90, rot180, rot270, flip-x,
    # flip-y, transpose, anti-transpose; anchors t in T0 order; duplicates
    # (as offset sets) keep their first enumeration index
    sym = [lambda x, y: (x, y), lambda x, y: (-y, x), lambda x, y: (-x, -y), lambda x, y: (y, -x),
           lambda x, y: (-x, y), lambda x, y: (x, -y), lambda x, y: (y, x), lambda x, y: (-y, -x)]
    t0 = [(a, b) for a in range(5) for b in range(5 - a)]
    seen, e = set(), 0
    for g in sym:
        for t in t0:
            offs = tuple(sorted(g(p[0] - t[0], p[1] - t[1]) for p in t0))
            if offs in seen:
                continue
            seen.add(offs)
            if all(feasible(dx, dy) for dx, dy in offs):
                ranked.append((key_of(offs) + (0, e), offs))
            e += 1
    # (b) line lattices along x (axis 0) and along y (axis 1): q's line and
    # four others within distance 4, holding a permutation of 5, 4, 3, 2, 1
    # cells, each line's feasible cells taken nearest-first (ties: negative
    # side first)
    along = sorted(range(-radius, radius + 1), key=lambda v: (abs(v), v))
    others = [d for d in range(-radius, radius + 1) if d != 0]
    for axis in (0, 1):
        e = 0
        for comb in itertools.combinations(others, 4):
            ls = sorted((0,) + comb)
            for counts in itertools.permutations((5, 4, 3, 2, 1)):
                offs, ok = [], True
                for d, k in zip(ls, counts):
                    cells = [((t, d) if axis == 0 else (d, t)) for t in along]
                    cells = [c for c in cells if feasible(*c)]
                    if len(cells) < k:
                        ok = False
                        break
                    offs += cells[:k]
                if ok:
                    ranked.append((key_of(offs) + (1 + axis, e), tuple(sorted(offs))))
                e += 1
    ranked.sort(key=lambda r: r[0])
    pool, seen = [], set()
    for _, offs in ranked:
        cells = tuple(sorted((qj + dy) * nx + qi + dx for dx, dy in offs))
        if cells not in seen:
            seen.add(cells)
            pool.append(list(cells))
            if len(pool) == pool_size:
                break
    return pool


@pytest.mark.parametrize("case", [1, 2, 4, 5, "P1", "P2N", "P3", "P3R"])
def test_lattice_pool_equals_brute_force_enumeration(case):
    """The oracle's R-PLG pool (keys computed by prefix sums over each
    line's cells, all candidates sorted, cell lists built in rank order)
    equals the rule enumerated directly, on the most constrained irregular
    cells of each case (fewest non-empty cells within distance 4) and on
    seeded random ones."""
    cfg = W.problem(case, 40 if case == "P1" else 64) if isinstance(case, str) else W.config(case, n=64)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    disc = Discretization(cg, cfg["a"], cfg["b"], cfg["c"], eager=False)
    irr = [int(q) for q in disc.irregular]
    nx, ny = disc.nx, disc.ny

    def k_size(q):
        qi, qj = q % nx, q // nx
        return sum(1 for dy in range(-4, 5) for dx in range(-4, 5)
                   if 0 <= qi + dx < nx and 0 <= qj + dy < ny and disc.nonempty[(qj + dy) * nx + qi + dx])

    tight = sorted(irr, key=lambda q: (k_size(q), q))[:3]
    rng = np.random.default_rng(77)
    sample = tight + [int(v) for v in rng.choice(irr, size=3, replace=False)]
    for q in sample:
        assert disc.lattice_pool(q) == _brute_force_pool(disc, q), q
