"""Spatial discretization for the oracle (Sections 2.2-2.3, 3.2-3.4).

* Regular cells (every cell of the 5x5 box S_Lap u S_Cro around them is pure,
  Section 3.2) use the fourth-order finite-volume formulas eq. stdLap for
  u_xx, u_yy and the iterated eq. stdGrad for u_xy.
* Irregular cells get a 15-cell poised lattice from the rule R-PLG below and
  weights from the weighted minimum-norm problem eq. derivedCoefAgain with the
  weights eq. weightDef and the recentred, scaled basis of Section 3.3.
* Assembly gives L u + N g = f (eq. PoissonLinearDiscretization); N holds one
  column per boundary face (cell, curve).

R-PLG (the paper cites its PLG algorithm without giving it; this is the
deterministic rule both implementations follow).  The feasible set K is every
non-empty cell within infinity-distance 4 of q.  Two families of 15-cell
lattices are considered, both poised for degree-4 polynomials:

  (a) images q + g(T0 - t) of the principal lattice T0 = {p >= 0, p1+p2 <= 4}
      for the eight symmetries g of the square and the 15 anchors t in T0;
  (b) line lattices: five distinct grid rows (or columns) within distance 4,
      one of them q's own, holding 5, 4, 3, 2 and 1 cells, each line taking
      its feasible cells nearest-first to q.  A polynomial of degree 4 that
      vanishes on such a set vanishes on the 5-cell line, then on the 4-cell
      line, and so on, so the set is poised: it is the principal lattice with
      every row shifted on its own.

Lattices inside K are ranked by (sum of squared distances to q, largest
infinity distance, family/axis, enumeration index), duplicates dropped, and
the 16 most compact are fitted.  A fit is acceptable when the 15x15
cell-average sample matrix has 2-norm condition number <= 1e8 and the cell's
own weight is at most -(a+c)/2 (in units of 1/h^2; the regular stencil has
-5(a+c)/2): a positive own weight makes the row anti-diffusive and gives the
operator spurious growing modes.  Among acceptable fits the one with the
smallest W^{-1}-norm of its weights is taken -- the quantity eq.
derivedCoefAgain minimises for a fixed lattice (norms within a relative 1e-9
count as equal; the earlier lattice wins).  No acceptable fit is a PLG
failure.

The least-squares problem is posed in grid-scaled coordinates xi = (x - p)/h:
the cell columns and L-hat are dimensionless, a Neumann column uses the
xi-gradient, and the weights are converted back by 1/h^2 (cells, Dirichlet
faces) and 1/h (Neumann faces).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .geometry import CUT, DEG, DIRICHLET, EMPTY, MERGED, NEUMANN, PURE, ROBIN, shift_moments

K_EMPTY, K_MERGED, K_REGULAR, K_IRR_PURE, K_IRR_CUT = 0, 1, 2, 3, 4
PLG_RADIUS = 4
COND_MAX = 1e8
PLG_POOL = 16        # most compact feasible lattices that are fitted
OWN_WEIGHT_MAX = -0.5  # own weight bound, in units of (a+c)/h^2
NORM_TIE = 1e-9

T0 = [(p1, p2) for p1 in range(5) for p2 in range(5 - p1)]
D4 = [
    lambda x, y: (x, y),       # identity
    lambda x, y: (-y, x),      # rotation by 90
    lambda x, y: (-x, -y),     # rotation by 180
    lambda x, y: (y, -x),      # rotation by 270
    lambda x, y: (-x, y),      # reflection x -> -x
    lambda x, y: (x, -y),      # reflection y -> -y
    lambda x, y: (y, x),       # transpose
    lambda x, y: (-y, -x),     # anti-transpose
]
# graded-lex basis exponents: degree 0..4, x power descending
BASIS = [(a, d - a) for d in range(DEG + 1) for a in range(d, -1, -1)]


class PLGError(Exception):
    pass


def ranked_candidates():
    """Offset sets of the principal-lattice images, deduplicated, in
    enumeration order (symmetry, then anchor)."""
    seen = set()
    cands = []
    for gi, g in enumerate(D4):
        for ti, t in enumerate(T0):
            offs = tuple(sorted(g(p[0] - t[0], p[1] - t[1]) for p in T0))
            if offs in seen:
                continue
            seen.add(offs)
            cands.append(offs)
    return cands


_CANDIDATES = ranked_candidates()
_CAND_OFFS = np.array(_CANDIDATES)                      # (n, 15, 2) offsets (dx, dy)
_CAND_SUMSQ = (_CAND_OFFS ** 2).sum(axis=(1, 2))
_CAND_MAX = np.abs(_CAND_OFFS).max(axis=(1, 2))


def _line_assignments():
    """(lines, counts) pairs of the second PLG stage in enumeration order: the
    line through q (offset 0) plus four of the eight others, the counts a
    permutation of (5, 4, 3, 2, 1)."""
    import itertools
    others = [d for d in range(-PLG_RADIUS, PLG_RADIUS + 1) if d != 0]
    out = []
    for comb in itertools.combinations(others, 4):
        lines = tuple(sorted((0,) + comb))
        for perm in itertools.permutations((5, 4, 3, 2, 1)):
            out.append((lines, perm))
    return out


_LINE_ASSIGN = _line_assignments()
_LINE_SETS = np.array([ls for ls, _ in _LINE_ASSIGN])
_LINE_COUNTS = np.array([cn for _, cn in _LINE_ASSIGN])
_ALONG = sorted(range(-PLG_RADIUS, PLG_RADIUS + 1), key=lambda v: (abs(v), v))


def regular_coefficients(a, b, c, h):
    """Regular-row stencil {(dx, dy): coefficient} (eq. stdLap, eq. stdGrad)."""
    s = 1.0 / (12.0 * h * h)
    co = {(0, 0): -30.0 * (a + c) * s}
    for m, w in ((1, 16.0), (2, -1.0)):
        for sg in (1, -1):
            co[(sg * m, 0)] = co.get((sg * m, 0), 0.0) + w * a * s
            co[(0, sg * m)] = co.get((0, sg * m), 0.0) + w * c * s
    if b != 0.0:
        g = {1: 8.0, 2: -1.0, -1: -8.0, -2: 1.0}
        for m1 in (-2, -1, 1, 2):
            for m2 in (-2, -1, 1, 2):
                co[(m1, m2)] = b * g[m1] * g[m2] / (144.0 * h * h)
    return co


class Discretization:
    """L and N of one grid level."""

    def __init__(self, cg, a, b, c, w_min=0.5, cond_max=COND_MAX, need_plg_parity=True, eager=True,
                 lattice_rule="min_norm"):
        """eager=False skips fitting the irregular rows; ``row(q)`` then fits
        one on demand (large grids sampled cell by cell).  lattice_rule:
        which acceptable lattice R-PLG keeps, "min_norm" (the smallest
        W^-1-norm of the weights; the library's rule) or "min_cond" (the
        smallest condition number of the cell sample matrix; a measured
        alternative, not used by the library)."""
        if b * b - 4.0 * a * c >= 0.0:
            raise ValueError("operator is not elliptic")
        if lattice_rule not in ("min_norm", "min_cond"):
            raise ValueError("unknown lattice rule %r" % lattice_rule)
        self.lattice_rule = lattice_rule
        self.cg = cg
        self.a, self.b, self.c = float(a), float(b), float(c)
        self.w_min = w_min
        self.cond_max = cond_max
        nx, ny = cg.nx, cg.ny
        self.nx, self.ny, self.h = nx, ny, cg.h
        st = cg.state.reshape(ny, nx)
        nonempty = (st == PURE) | (st == CUT)
        pure = st == PURE
        pp = np.zeros((ny + 4, nx + 4), dtype=bool)
        pp[2:-2, 2:-2] = pure
        reg = np.ones((ny, nx), dtype=bool)
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                reg &= pp[2 + dy:2 + dy + ny, 2 + dx:2 + dx + nx]
        reg &= nonempty
        kind = np.zeros((ny, nx), dtype=np.int8)
        kind[st == MERGED] = K_MERGED
        kind[reg] = K_REGULAR
        kind[nonempty & ~reg & pure] = K_IRR_PURE
        kind[nonempty & ~reg & ~pure] = K_IRR_CUT
        self.kind = kind.ravel()
        self.nonempty = nonempty.ravel()
        self.regular = reg.ravel()
        self.irregular = np.flatnonzero(self.nonempty & ~self.regular)
        self.coef = regular_coefficients(self.a, self.b, self.c, self.h)
        self.diag = self.coef[(0, 0)]
        # boundary faces, ordered by (cell, curve)
        self.faces = []
        for idx in self.irregular:
            for cv in sorted(cg.faces(int(idx))):
                self.faces.append((int(idx), cv))
        self.face_index = {f: k for k, f in enumerate(self.faces)}
        self._pure_cache = {}
        self.stencils = {}
        self.weights = {}
        self.face_weights = {}
        self.conds = {}
        if eager:
            for idx in self.irregular:
                self._row(int(idx))

    def row(self, q):
        """Lattice, weights and face weights of irregular cell q (fitted on
        first use)."""
        if q not in self.stencils:
            self._row(q)
        return self.stencils[q], self.weights[q], self.face_weights.get(q, [])

    # -- averages of basis functions -----------------------------------------
    def _cell_offset(self, k, p):
        return (k % self.nx + 0.5 - p[0], k // self.nx + 0.5 - p[1])

    def basis_averages(self, k, p):
        """<phi_alpha>_k for the scaled basis about p (grid units)."""
        d, e = self._cell_offset(k, p)
        pure = self.cg.state[k] == PURE
        if pure and (d, e) in self._pure_cache:
            return self._pure_cache[(d, e)]
        m = shift_moments(self.cg.moments(k), d, e)
        vol = m[0, 0]
        out = np.array([m[a1, a2] / vol for a1, a2 in BASIS])
        if pure:
            self._pure_cache[(d, e)] = out
        return out

    def operator_averages(self, k, p):
        """<L_xi phi_alpha>_k, L_xi = a d_xx + b d_xy + c d_yy in scaled units."""
        d, e = self._cell_offset(k, p)
        m = shift_moments(self.cg.moments(k), d, e)
        vol = m[0, 0]
        out = []
        for a1, a2 in BASIS:
            v = 0.0
            if a1 >= 2:
                v += self.a * a1 * (a1 - 1) * m[a1 - 2, a2]
            if a1 >= 1 and a2 >= 1:
                v += self.b * a1 * a2 * m[a1 - 1, a2 - 1]
            if a2 >= 2:
                v += self.c * a2 * (a2 - 1) * m[a1, a2 - 2]
            out.append(v / vol)
        return np.array(out)

    def face_column(self, k, face, p):
        """<<N phi_alpha>> over a boundary face of cell k: Dirichlet averages the
        basis, Neumann averages its xi-gradient along the outward normal, Robin
        (gamma1 + gamma2 d/dn, Section 3) is the face average of N phi divided
        by s = |gamma1| + |gamma2| / h (robin_scale), which keeps the column
        O(1) and makes it the Dirichlet column for gamma2 = 0 and the Neumann
        one for gamma1 = 0."""
        d, e = self._cell_offset(k, p)
        L = face.length
        curve = self.cg.curves[face.curve]
        bc = curve.bc
        if bc == ROBIN:
            g1, g2 = curve.robin
            dcol = self._face_dirichlet(face, d, e)
            ncol = self._face_normal(face, d, e)
            return (g1 * dcol + (g2 / self.h) * ncol) / self.robin_scale(curve)
        if bc == DIRICHLET:
            return self._face_dirichlet(face, d, e)
        return self._face_normal(face, d, e)

    def robin_scale(self, curve):
        """s = |gamma1| + |gamma2| / h: the Robin column is N phi / s."""
        g1, g2 = curve.robin
        return abs(g1) + abs(g2) / self.h

    def _face_dirichlet(self, face, d, e):
        m = shift_moments(face.m, d, e)
        return np.array([m[a1, a2] / face.length for a1, a2 in BASIS])

    def _face_normal(self, face, d, e):
        L = face.length
        mx = shift_moments(face.mx, d, e)
        my = shift_moments(face.my, d, e)
        out = []
        for a1, a2 in BASIS:
            v = 0.0
            if a1 >= 1:
                v += a1 * mx[a1 - 1, a2]
            if a2 >= 1:
                v += a2 * my[a1, a2 - 1]
            out.append(v / L)
        return np.array(out)

    # -- R-PLG -----------------------------------------------------------------
    def _feasible(self, i, j):
        return 0 <= i < self.nx and 0 <= j < self.ny and self.nonempty[j * self.nx + i]

    def lattice_pool(self, q):
        """The PLG_POOL most compact feasible lattices (sorted cell lists).

        Every candidate of both families that lies inside K is ranked by
        (sum of squared distances to q, largest infinity distance,
        family/axis, enumeration index); the candidates are taken in that
        order, duplicates dropped, until PLG_POOL distinct lattices are
        found.  The keys of all candidates are computed (and sorted) before
        any is taken; only the cell lists are built on demand, in rank order.

        Parity unpinned: the paper does not give its PLG algorithm, so which
        poised lattice is chosen is this project's rule (module docstring);
        tests pin only what any valid choice satisfies (15 distinct cells
        inside K, containing q, poised, exactness of the fitted row) and that
        this pool equals a brute-force enumeration of the rule."""
        nx = self.nx
        qi, qj = q % nx, q // nx
        R = PLG_RADIUS
        win = np.zeros((2 * R + 1, 2 * R + 1), dtype=bool)   # win[dy + R, dx + R]
        for dy in range(-R, R + 1):
            for dx in range(-R, R + 1):
                win[dy + R, dx + R] = self._feasible(qi + dx, qj + dy)
        # (a) images of the principal lattice: feasibility and keys
        ok = np.flatnonzero(np.all(win[_CAND_OFFS[:, :, 1] + R, _CAND_OFFS[:, :, 0] + R], axis=1))
        keys = [(_CAND_SUMSQ[ok], _CAND_MAX[ok], np.zeros(ok.size, dtype=np.int64), ok)]
        # (b) line lattices: on line d (offset d across the axis) the feasible
        # cells nearest-first; taking the first k of them costs
        # cost[d, k] = sum of their squared distances and reaches reach[d, k]
        lines = {}
        for axis in (0, 1):
            avail = np.zeros(2 * R + 1, dtype=np.int64)
            cost = np.zeros((2 * R + 1, 6), dtype=np.int64)
            reach = np.zeros((2 * R + 1, 6), dtype=np.int64)
            for d in range(-R, R + 1):
                cl = []
                for t in _ALONG:
                    dx, dy = (t, d) if axis == 0 else (d, t)
                    if win[dy + R, dx + R]:
                        cl.append((t, (qj + dy) * nx + qi + dx))
                lines[(axis, d)] = cl
                avail[d + R] = len(cl)
                for k in range(1, min(5, len(cl)) + 1):
                    t = cl[k - 1][0]
                    cost[d + R, k] = cost[d + R, k - 1] + t * t + d * d
                    reach[d + R, k] = max(reach[d + R, k - 1], abs(t), abs(d))
            feas = np.flatnonzero(np.all(avail[_LINE_SETS + R] >= _LINE_COUNTS, axis=1))
            tot = cost[_LINE_SETS[feas] + R, _LINE_COUNTS[feas]].sum(axis=1)
            mx = reach[_LINE_SETS[feas] + R, _LINE_COUNTS[feas]].max(axis=1)
            keys.append((tot, mx, np.full(feas.size, 1 + axis, dtype=np.int64), feas))
        sumsq, mxd, fam, enum = (np.concatenate([k[i] for k in keys]) for i in range(4))
        order = np.lexsort((enum, fam, mxd, sumsq))

        def cells_of(f, e):
            if f == 0:
                return sorted((qj + dy) * nx + qi + dx for dx, dy in _CANDIDATES[e])
            out = []
            for d, k in zip(_LINE_SETS[e], _LINE_COUNTS[e]):
                out += [c for _, c in lines[(f - 1, int(d))][:int(k)]]
            return sorted(out)

        pool, seen = [], set()
        for r in order:
            cells = cells_of(int(fam[r]), int(enum[r]))
            key = tuple(cells)
            if key not in seen:
                seen.add(key)
                pool.append(cells)
                if len(pool) == PLG_POOL:
                    break
        return pool

    def fit(self, q, cells):
        """Weighted minimum-norm weights (scaled units) of lattice ``cells``
        plus q's boundary faces; returns (cond, beta, face keys, w)."""
        faces = self.cg.faces(q)
        fkeys = sorted(faces)
        p = self._bbox_centre(cells)
        cols = [self.basis_averages(k, p) for k in cells]
        cond = np.linalg.cond(np.array(cols).T)
        cols += [self.face_column(q, faces[f], p) for f in fkeys]
        M = np.array(cols).T                        # N x (N + nf)
        Lhat = self.operator_averages(q, p)
        qi, qj = q % self.nx, q // self.nx
        w = [max(math.hypot(k % self.nx - qi, k // self.nx - qj), self.w_min) for k in cells]
        w += [self.w_min] * len(fkeys)
        w = np.array(w)
        return cond, weighted_min_norm(M, w, Lhat), fkeys, w

    def plg(self, q):
        """R-PLG: lattice and weights for irregular cell q.

        Parity unpinned as to the choice of lattice (see lattice_pool); the
        weights of a given lattice are pinned (exact rationals, exactness on
        quartics, agreement with the minimum-norm characterisation)."""
        best = None
        bound = OWN_WEIGHT_MAX * (self.a + self.c)
        for cells in self.lattice_pool(q):
            cond, beta, fkeys, w = self.fit(q, cells)
            if cond > self.cond_max or beta[cells.index(q)] > bound:
                continue
            nrm = float(np.sum(w * beta * beta)) if self.lattice_rule == "min_norm" else cond
            if best is None or nrm < best[0] * (1.0 - NORM_TIE):
                best = (nrm, cells, cond, beta, fkeys)
        if best is None:
            raise PLGError("no acceptable lattice for cell %d" % q)
        return best[1:]

    def _bbox_centre(self, cells):
        ii = [k % self.nx for k in cells]
        jj = [k // self.nx for k in cells]
        return (0.5 * (min(ii) + max(ii) + 1), 0.5 * (min(jj) + max(jj) + 1))

    # -- weighted minimum-norm weights (eq. derivedCoefAgain) -------------------
    def _row(self, q):
        cells, cond, beta, fkeys = self.plg(q)
        self.stencils[q] = cells
        self.conds[q] = cond
        h = self.h
        self.weights[q] = beta[:len(cells)] / (h * h)
        fw = []
        for f, bf in zip(fkeys, beta[len(cells):]):
            # the Neumann column is in xi-gradient units (h du/dn), the
            # Dirichlet column in the datum's units, the Robin column the
            # datum divided by s
            curve = self.cg.curves[f]
            if curve.bc == NEUMANN:
                w = bf / h
            elif curve.bc == ROBIN:
                w = bf / (self.robin_scale(curve) * h * h)
            else:
                w = bf / (h * h)
            fw.append((self.face_index[(q, f)], w))
        self.face_weights[q] = fw

    # -- assembly ----------------------------------------------------------------
    def matrices(self):
        """Sparse L (n x n, grid-indexed) and N (n x n_faces)."""
        nx, ny = self.nx, self.ny
        n = nx * ny
        rows, cols, vals = [], [], []
        reg = np.flatnonzero(self.regular)
        ri, rj = reg % nx, reg // nx
        for (dx, dy), v in self.coef.items():
            rows.append(reg)
            cols.append((rj + dy) * nx + ri + dx)
            vals.append(np.full(reg.size, v))
        for q in self.irregular:
            q = int(q)
            rows.append(np.full(15, q))
            cols.append(np.array(self.stencils[q]))
            vals.append(self.weights[q])
        L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        nr, nc, nv = [], [], []
        for q in self.irregular:
            for fk, v in self.face_weights[int(q)]:
                nr.append(int(q))
                nc.append(fk)
                nv.append(v)
        N = sp.csr_matrix((nv, (nr, nc)), shape=(n, max(1, len(self.faces))))
        return L, N

    def irregular_rows(self):
        """CSR of the irregular rows only: (row cell, cols, vals)."""
        return {int(q): (np.array(self.stencils[int(q)]), self.weights[int(q)]) for q in self.irregular}

    def apply(self, u, g=None):
        """(L u)_i (+ (N g)_i) on every non-empty cell; u grid-shaped or flat.

        Regular rows use the difference form sum_m c_m (u_{i+m} - u_i), an exact
        rewrite because the stencil coefficients sum to zero."""
        nx, ny = self.nx, self.ny
        U = np.asarray(u, dtype=float).reshape(ny, nx)
        out = np.zeros((ny, nx))
        P = np.zeros((ny + 4, nx + 4))
        P[2:-2, 2:-2] = U
        acc = np.zeros((ny, nx))
        for (dx, dy), v in self.coef.items():
            if dx == 0 and dy == 0:
                continue
            acc += v * (P[2 + dy:2 + dy + ny, 2 + dx:2 + dx + nx] - U)
        out[self.regular.reshape(ny, nx)] = acc[self.regular.reshape(ny, nx)]
        flat = out.ravel()
        uf = U.ravel()
        for q in self.irregular:
            q = int(q)
            cols = self.stencils[q]
            flat[q] = float(np.dot(self.weights[q], uf[cols]))
            if g is not None:
                for fk, v in self.face_weights[q]:
                    flat[q] += v * g[fk]
        return flat.reshape(ny, nx)


def weighted_min_norm(M, w, Lhat):
    """beta = W M^T (M W M^T)^{-1} Lhat with W^{-1} = diag(w) (Prop. leastSquares
    (ii), eq. derivedCoefAgain), evaluated through a QR factorisation of
    W^{1/2} M^T so that the normal matrix is never formed."""
    s = 1.0 / np.sqrt(w)
    A = s[:, None] * M.T
    Q, R = np.linalg.qr(A)
    y = np.linalg.solve(R.T, Lhat)
    return s * (Q @ y)


def discretize(cg, a, b, c, **kw):
    return Discretization(cg, a, b, c, **kw)


def boundary_data(disc, sol, q=16):
    """g-hat: face averages of N u for every face: u (Dirichlet), du/dn
    (Neumann) or gamma1 u + gamma2 du/dn (Robin, the boundary operator of
    Section 3)."""
    from .geometry import face_averages
    g = np.zeros(max(1, len(disc.faces)))
    cache = {}
    for k, (idx, curve) in enumerate(disc.faces):
        if idx not in cache:
            cache[idx] = face_averages(disc.cg, idx, sol.u, sol.dudn, q=q)
        g[k] = cache[idx][curve]
    return g
