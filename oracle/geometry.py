"""Cut-cell geometry for the oracle (Section 3.1 and Alg. 1; cubature of
Section 2.4).

Reading of the paper used here (the paper represents domains as Yin sets with
spline boundaries; the workloads here use analytic curves instead):

* Grid cells are C_ij = (x0+ih, x0+(i+1)h) x (y0+jh, y0+(j+1)h); the cut cell
  is C_ij intersected with the open domain, the cut face likewise, and the
  boundary piece S_ij is taken on the *closure* of the cell, so cells whose
  edge lies on the outer box own that edge as a boundary piece.
* Each analytic curve is split at the parameters where x'(t) or y'(t)
  vanishes, so every piece is monotone in both coordinates; crossings with the
  grid lines are found by bisection inside each piece.  The resulting sub-arcs
  each lie in one cell.
* The boundary of a cut cell is traced as loops: follow an arc (oriented with
  the domain on its left) to its exit point on the cell perimeter, then walk
  the perimeter counter-clockwise to the next entry point.  Each loop bounds
  one connected component.
* Volumes and moments use Green's formula with the x-primitive (eq.
  volumeIntegral / iteratedIntegral): vertical cell edges integrate exactly,
  horizontal edges contribute nothing, arcs use Gauss-Legendre in the curve
  parameter.  Moments are taken in grid-scaled coordinates
  X = (x - c_x)/h, Y = (y - c_y)/h about the cell centre c.
* Alg. 1: every extra connected component of a cell is moved to the edge
  neighbour with which it shares the longest stretch of cell edge; then, in
  increasing linear index with live volumes, each interface cell with volume
  <= theta h^2 is merged into the non-empty edge neighbour with the longest
  common cut face (ties in the order -x, +x, -y, +y).  Lengths within
  MERGE_TIE (units of h) of each other are ties: faces of equal length in
  exact arithmetic (the two legs of a corner triangle cut by a 45-degree
  edge) come out of the crossing search a few ulps apart, and rounding must
  not decide between them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BOX, CIRCLE, ELLIPSE, POLAR_SIN, POLAR_COS, POLYGON = 0, 1, 2, 3, 4, 5
QUARTER = 0.5 * math.pi   # parameter length of one polygon edge
DIRICHLET, NEUMANN, ROBIN = 0, 1, 2
TWO_PI = 2.0 * math.pi
GL_Q = 16                 # Gauss-Legendre nodes per arc piece
DEG = 4                   # moments up to total degree 4
POLAR_SAMPLES = 8192      # derivative sampling for polar-curve extrema
DEGENERATE_CHORD = 1e-10  # sub-arcs shorter than this (in units of h) are dropped
PERIM_SNAP = 1e-9         # perimeter gaps below this are read as touching
EXTREMUM_REL = 1e-8       # |x'(t)| (or |y'(t)|) below this times |c'(t)|: an extremum of x (or y)
MERGE_TIE = 1e-12         # cut-face lengths (units of h) within this of each other tie in Alg. 1

# cell states after Alg. 1
EMPTY, MERGED, PURE, CUT = 0, 1, 2, 3


class GeometryError(Exception):
    pass


_GL_CACHE = {}


def gauss_legendre(q):
    """Nodes and weights on [-1, 1] (library routine)."""
    if q not in _GL_CACHE:
        _GL_CACHE[q] = np.polynomial.legendre.leggauss(q)
    return _GL_CACHE[q]


# ---------------------------------------------------------------------------
# Curves
# ---------------------------------------------------------------------------
class Curve:
    def __init__(self, desc, index):
        self.kind = int(desc["kind"])
        self.p = [float(v) for v in desc["p"]]
        self.inside = int(desc["inside"])
        self.bc = int(desc["bc"])
        # Robin: gamma1 u + gamma2 du/dn (the boundary operator N of Section 3)
        self.robin = tuple(float(v) for v in desc.get("robin", (0.0, 0.0)))
        self.index = index

    def datum(self, fn_value, fn_normal, px, py, nx, ny):
        """N u at a boundary point: u (Dirichlet), du/dn (Neumann) or
        gamma1 u + gamma2 du/dn (Robin); n is the outward normal of the domain."""
        if self.bc == DIRICHLET:
            return fn_value(px, py)
        if self.bc == NEUMANN:
            return fn_normal(px, py, nx, ny)
        return self.robin[0] * fn_value(px, py) + self.robin[1] * fn_normal(px, py, nx, ny)

    # r(t) for polar curves
    def _r(self, t):
        cx, cy, r0, A, k, ph = self.p
        if self.kind == POLAR_SIN:
            return r0 + A * math.sin(k * t + ph), A * k * math.cos(k * t + ph)
        return r0 + A * math.cos(k * t + ph), -A * k * math.sin(k * t + ph)

    # polygon: a convex quadrilateral, vertices counter-clockwise in p;
    # edge k is traversed for t in [k pi/2, (k+1) pi/2)
    def _edge(self, t):
        k = min(3, max(0, int(math.floor((t % TWO_PI) / QUARTER))))
        s = (t % TWO_PI) / QUARTER - k
        v = self.p
        ax, ay = v[2 * k], v[2 * k + 1]
        bx, by = v[(2 * k + 2) % 8], v[(2 * k + 3) % 8]
        return ax, ay, bx, by, s

    def point(self, t):
        if self.kind == POLYGON:
            ax, ay, bx, by, s = self._edge(t)
            return ax + s * (bx - ax), ay + s * (by - ay)
        if self.kind == CIRCLE:
            cx, cy, r = self.p
            return cx + r * math.cos(t), cy + r * math.sin(t)
        if self.kind == ELLIPSE:
            cx, cy, a1, a2, rot = self.p
            u, v = a1 * math.cos(t), a2 * math.sin(t)
            cr, sr = math.cos(rot), math.sin(rot)
            return cx + cr * u - sr * v, cy + sr * u + cr * v
        cx, cy = self.p[0], self.p[1]
        r, _ = self._r(t)
        return cx + r * math.cos(t), cy + r * math.sin(t)

    def deriv(self, t):
        if self.kind == POLYGON:
            ax, ay, bx, by, _ = self._edge(t)
            return (bx - ax) / QUARTER, (by - ay) / QUARTER
        if self.kind == CIRCLE:
            r = self.p[2]
            return -r * math.sin(t), r * math.cos(t)
        if self.kind == ELLIPSE:
            cx, cy, a1, a2, rot = self.p
            du, dv = -a1 * math.sin(t), a2 * math.cos(t)
            cr, sr = math.cos(rot), math.sin(rot)
            return cr * du - sr * dv, sr * du + cr * dv
        r, dr = self._r(t)
        c, s = math.cos(t), math.sin(t)
        return dr * c - r * s, dr * s + r * c

    def contains(self, x, y):
        """Strictly inside the closed curve (the curve itself is outside)."""
        if self.kind == POLYGON:
            v = self.p
            for k in range(4):
                ax, ay, bx, by = v[2 * k], v[2 * k + 1], v[(2 * k + 2) % 8], v[(2 * k + 3) % 8]
                if (bx - ax) * (y - ay) - (by - ay) * (x - ax) <= 0.0:
                    return False
            return True
        if self.kind == CIRCLE:
            cx, cy, r = self.p
            return (x - cx) ** 2 + (y - cy) ** 2 < r * r
        if self.kind == ELLIPSE:
            cx, cy, a1, a2, rot = self.p
            cr, sr = math.cos(rot), math.sin(rot)
            dx, dy = x - cx, y - cy
            u = cr * dx + sr * dy
            v = -sr * dx + cr * dy
            return (u / a1) ** 2 + (v / a2) ** 2 < 1.0
        cx, cy = self.p[0], self.p[1]
        dx, dy = x - cx, y - cy
        rho = math.hypot(dx, dy)
        r, _ = self._r(math.atan2(dy, dx))
        return rho < r

    def breakpoints(self):
        """Parameters in [0, 2 pi) where x'(t) = 0 or y'(t) = 0 (polygon: its
        vertices, where x' and y' jump)."""
        if self.kind == POLYGON:
            return [0.0, QUARTER, 2 * QUARTER, 3 * QUARTER]
        if self.kind == CIRCLE:
            return [0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi]
        if self.kind == ELLIPSE:
            cx, cy, a1, a2, rot = self.p
            cr, sr = math.cos(rot), math.sin(rot)
            tx = math.atan2(-a2 * sr, a1 * cr)
            ty = math.atan2(a2 * cr, a1 * sr)
            ts = [tx, tx + math.pi, ty, ty + math.pi]
            return _dedupe(sorted(t % TWO_PI for t in ts))
        out = []
        S = POLAR_SAMPLES
        for comp in (0, 1):
            def g(t):
                return self.deriv(t)[comp]
            prev_t, prev_v = 0.0, g(0.0)
            for s in range(1, S + 1):
                t = TWO_PI * s / S
                v = g(t)
                if prev_v == 0.0:
                    out.append(prev_t)
                elif prev_v * v < 0.0:
                    out.append(_bisect_sign(g, prev_t, t))
                prev_t, prev_v = t, v
        return _dedupe(sorted(t % TWO_PI for t in out))

    def extent(self):
        """Axis-aligned bounding box from the extrema."""
        pts = [self.point(t) for t in self.breakpoints()]
        xs = [p[0] for p in pts]
        ys = [p[1] for p in pts]
        return min(xs), max(xs), min(ys), max(ys)


def _dedupe(ts):
    out = []
    for t in ts:
        if not out or t - out[-1] > 1e-14:
            out.append(t)
    if len(out) > 1 and out[0] + TWO_PI - out[-1] <= 1e-14:
        out.pop()
    return out


def _bisect_sign(g, lo, hi):
    glo = g(lo)
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        gm = g(mid)
        if gm == 0.0:
            return mid
        if (gm < 0.0) == (glo < 0.0):
            lo, glo = mid, gm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _bisect_level(fn, lo, hi, level):
    """Root of the monotone function fn(t) - level on [lo, hi]."""
    flo = fn(lo) - level
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        fm = fn(mid) - level
        if fm == 0.0:
            return mid
        if (fm < 0.0) == (flo < 0.0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------------------
# Data records
# ---------------------------------------------------------------------------
@dataclass
class CellArc:
    """A maximal run of a curve inside one cell, oriented with the domain on
    its left.  ``pieces`` are parameter intervals in the curve's own (ccw)
    direction; ``sigma`` = +1 keeps that direction, -1 reverses it."""
    curve: int
    sigma: int
    pieces: list
    p_in: tuple
    p_out: tuple
    s_in: float = 0.0
    s_out: float = 0.0


@dataclass
class Face:
    """Moments of a boundary piece (one curve) in scaled coordinates about a
    centre: length, m[a,b] = int X^a Y^b ds, mx/my = int X^a Y^b n_x|n_y ds."""
    curve: int
    length: float = 0.0
    m: np.ndarray = field(default_factory=lambda: np.zeros((DEG + 1, DEG + 1)))
    mx: np.ndarray = field(default_factory=lambda: np.zeros((DEG + 1, DEG + 1)))
    my: np.ndarray = field(default_factory=lambda: np.zeros((DEG + 1, DEG + 1)))

    def copy(self):
        return Face(self.curve, self.length, self.m.copy(), self.mx.copy(), self.my.copy())


@dataclass
class Component:
    """One connected component of a cut cell, moments about its own cell centre."""
    cell: int
    mom: np.ndarray               # mom[a,b] = iint X^a Y^b dXdY  (a+b <= 4)
    edge_len: list                # inside length on edges (bottom, right, top, left)
    faces: dict                   # curve index -> Face
    loop: list = None             # the boundary loop it was traced from

    @property
    def volume(self):
        return float(self.mom[0, 0])


@dataclass
class ControlVolume:
    """A non-empty cell after merging: the union of its member components,
    moments and boundary faces shifted to the host cell centre."""
    idx: int
    members: list                 # (grid idx of the member's own cell, Component)
    mom: np.ndarray
    faces: dict

    @property
    def volume(self):
        return float(self.mom[0, 0])


def _shift_matrix(d):
    """S[a, p] = C(a, p) d^(a-p): (X + d)^a = sum_p S[a, p] X^p."""
    S = np.zeros((DEG + 1, DEG + 1))
    for a in range(DEG + 1):
        for p in range(a + 1):
            S[a, p] = math.comb(a, p) * d ** (a - p)
    return S


def shift_moments(m, d, e):
    """Moments about a centre moved by (d, e) cells (X' = X + d, Y' = Y + e):
    m'[a, b] = sum_{p<=a, q<=b} C(a,p) C(b,q) d^(a-p) e^(b-q) m[p, q].
    Entries with a + b > 4 are not defined and are set to zero."""
    out = _shift_matrix(d) @ m @ _shift_matrix(e).T
    out[_HIGH] = 0.0
    return out


_HIGH = np.add.outer(np.arange(DEG + 1), np.arange(DEG + 1)) > DEG


def square_moments():
    """Closed form iint_{[-1/2,1/2]^2} X^a Y^b."""
    def I(a):
        return (0.5 ** (a + 1) - (-0.5) ** (a + 1)) / (a + 1)
    m = np.zeros((DEG + 1, DEG + 1))
    for a in range(DEG + 1):
        for b in range(DEG + 1 - a):
            m[a, b] = I(a) * I(b)
    return m


# ---------------------------------------------------------------------------
# Grid + curve intersection
# ---------------------------------------------------------------------------
def perimeter_coord(X, Y):
    """Counter-clockwise perimeter coordinate s in [0, 4) of a point on the
    boundary of the unit cell (local corner-origin coordinates)."""
    d = [abs(Y), abs(1.0 - X), abs(1.0 - Y), abs(X)]
    e = min(range(4), key=lambda k: d[k])
    cl = lambda v: min(1.0, max(0.0, v))  # noqa: E731
    if e == 0:
        s = cl(X)
    elif e == 1:
        s = 1.0 + cl(Y)
    elif e == 2:
        s = 2.0 + (1.0 - cl(X))
    else:
        s = 3.0 + (1.0 - cl(Y))
    return s % 4.0


class CutGrid:
    """Cut cells of one grid level after Alg. 1."""

    def __init__(self, grid, curves, theta=0.3, q=GL_Q):
        self.x0, self.y0 = float(grid["x0"]), float(grid["y0"])
        self.h = float(grid["h"])
        self.nx, self.ny = int(grid["nx"]), int(grid["ny"])
        self.theta = theta
        self.q = q
        self.curves = [Curve(c, k) for k, c in enumerate(curves)]
        self._validate()
        self._intersect()
        self._classify_native()
        self._merge()

    # -- set-up ------------------------------------------------------------
    def _validate(self):
        xl, yl = self.x0, self.y0
        xr, yr = self.x0 + self.nx * self.h, self.y0 + self.ny * self.h
        outer = [c for c in self.curves if c.inside]
        if len(outer) > 1:
            raise GeometryError("more than one outer boundary")
        self.box = None
        for c in self.curves:
            if c.kind == BOX:
                if not c.inside:
                    raise GeometryError("a box must be the outer boundary")
                x0, y0, x1, y1 = c.p
                if not (abs(x0 - xl) <= 1e-12 and abs(y0 - yl) <= 1e-12 and abs(x1 - xr) <= 1e-12
                        and abs(y1 - yr) <= 1e-12):
                    raise GeometryError("the box must coincide with the grid extent")
                self.box = c
            else:
                ex = c.extent()
                if not (ex[0] > xl and ex[1] < xr and ex[2] > yl and ex[3] < yr):
                    raise GeometryError("curve %d leaves the grid" % c.index)
        if not outer:
            raise GeometryError("no outer boundary")

    def in_domain(self, x, y):
        for c in self.curves:
            if c.kind == BOX:
                continue
            if c.inside and not c.contains(x, y):
                return False
            if not c.inside and c.contains(x, y):
                return False
        return True

    def _intersect(self):
        """Split every curve into sub-arcs lying in single cells."""
        h, x0, y0 = self.h, self.x0, self.y0
        self.cell_arcs = {}
        for c in self.curves:
            if c.kind == BOX:
                continue
            bps = c.breakpoints()
            events = []      # (t, point)
            for b, tb in enumerate(bps):
                events.append((tb, c.point(tb)))
            nb = len(bps)
            for b in range(nb):
                ta = bps[b]
                tb = bps[b + 1] if b + 1 < nb else bps[0] + TWO_PI
                pa, pb = c.point(ta), c.point(tb)
                # grid lines strictly between the piece's end values; a line
                # within DEGENERATE_CHORD h of an end where this coordinate is
                # extremal only touches the curve (tangency) and is not
                # crossed -- on both pieces meeting there, so the reading is
                # consistent
                da, db = c.deriv(ta), c.deriv(tb)
                for comp, org in ((0, x0), (1, y0)):
                    lo, hi = min(pa[comp], pb[comp]), max(pa[comp], pb[comp])
                    ext = [pe[comp] for pe, de in ((pa, da), (pb, db))
                           if abs(de[comp]) <= EXTREMUM_REL * math.hypot(de[0], de[1])]
                    k0 = math.floor((lo - org) / h)
                    k1 = math.ceil((hi - org) / h)
                    for k in range(k0, k1 + 1):
                        xk = org + k * h
                        if not (lo < xk < hi):
                            continue
                        if any(abs(xk - v) <= DEGENERATE_CHORD * h for v in ext):
                            continue
                        t = _bisect_level(lambda tt, comp=comp: c.point(tt)[comp], ta, tb, xk)
                        p = c.point(t)
                        p = (xk, p[1]) if comp == 0 else (p[0], xk)
                        events.append((t, p))
            events.sort(key=lambda e: e[0])
            t_start = events[0][0]
            events.append((events[0][0] + TWO_PI, events[0][1]))
            # sub-arcs
            subs = []
            for e in range(len(events) - 1):
                ta, pa = events[e]
                tb, pb = events[e + 1]
                if math.hypot(pb[0] - pa[0], pb[1] - pa[1]) <= DEGENERATE_CHORD * h:
                    continue
                xm, ym = c.point(0.5 * (ta + tb))
                i = math.floor((xm - x0) / h)
                j = math.floor((ym - y0) / h)
                subs.append(((i, j), ta, tb, pa, pb))
            if not subs:
                raise GeometryError("curve %d is degenerate" % c.index)
            cellset = {s[0] for s in subs}
            if len(cellset) == 1:
                raise GeometryError("curve %d lies inside a single cell" % c.index)
            # rotate so that the list starts at a cell change
            start = 0
            while subs[start][0] == subs[start - 1][0]:
                start += 1
            subs = subs[start:] + subs[:start]
            runs = []
            for s in subs:
                if runs and runs[-1][0] == s[0]:
                    runs[-1][1].append(s)
                else:
                    runs.append([s[0], [s]])
            for (i, j), lst in runs:
                if not (0 <= i < self.nx and 0 <= j < self.ny):
                    raise GeometryError("curve %d leaves the grid" % c.index)
                pieces = [(s[1], s[2]) for s in lst]
                p_first, p_last = lst[0][3], lst[-1][4]
                if c.inside:
                    arc = CellArc(c.index, +1, pieces, p_first, p_last)
                else:
                    arc = CellArc(c.index, -1, pieces, p_last, p_first)
                xi, yj = x0 + i * h, y0 + j * h
                arc.s_in = perimeter_coord((arc.p_in[0] - xi) / h, (arc.p_in[1] - yj) / h)
                arc.s_out = perimeter_coord((arc.p_out[0] - xi) / h, (arc.p_out[1] - yj) / h)
                self.cell_arcs.setdefault(j * self.nx + i, []).append(arc)
        self.t_start = None

    # -- components --------------------------------------------------------
    def _loops(self, idx):
        arcs = sorted(self.cell_arcs[idx], key=lambda a: (a.s_in, a.curve, a.pieces[0][0]))
        used = [False] * len(arcs)
        loops = []
        for st in range(len(arcs)):
            if used[st]:
                continue
            loop = []
            a = st
            while True:
                used[a] = True
                so = arcs[a].s_out
                best, bd = None, None
                for b in range(len(arcs)):
                    d = arcs[b].s_in - so
                    if d < 0.0:
                        d += 4.0
                    if d > 4.0 - PERIM_SNAP:
                        d = 0.0
                    if bd is None or d < bd:
                        best, bd = b, d
                loop.append(("arc", arcs[a]))
                loop.append(("perim", so, so + bd))
                if best == st:
                    break
                if used[best]:
                    raise GeometryError("inconsistent boundary in cell %d" % idx)
                a = best
            loops.append(loop)
        return loops

    def _component(self, idx, loop):
        """Green's-formula moments of one loop about the cell centre."""
        h = self.h
        i, j = idx % self.nx, idx // self.nx
        cx, cy = self.x0 + (i + 0.5) * h, self.y0 + (j + 0.5) * h
        mom = np.zeros((DEG + 1, DEG + 1))
        edge_len = [0.0, 0.0, 0.0, 0.0]
        faces = {}
        tq, wq = gauss_legendre(self.q)
        for item in loop:
            if item[0] == "arc":
                arc = item[1]
                c = self.curves[arc.curve]
                f = faces.setdefault(arc.curve, Face(arc.curve))
                for ta, tb in arc.pieces:
                    half = 0.5 * (tb - ta)
                    mid = 0.5 * (ta + tb)
                    for qn in range(self.q):
                        t = mid + half * tq[qn]
                        w = wq[qn] * half
                        px, py = c.point(t)
                        dx, dy = c.deriv(t)
                        X, Y = (px - cx) / h, (py - cy) / h
                        dY = arc.sigma * dy / h        # dY/dt along the oriented arc
                        speed = math.hypot(dx, dy) / h  # ds/dt in units of h
                        nxds = arc.sigma * dy / h       # n_x ds/dt
                        nyds = -arc.sigma * dx / h      # n_y ds/dt
                        f.length += w * speed
                        for a in range(DEG + 1):
                            Xa = X ** a
                            for b in range(DEG + 1 - a):
                                Yb = Y ** b
                                mom[a, b] += w * X ** (a + 1) / (a + 1) * Yb * dY
                                f.m[a, b] += w * Xa * Yb * speed
                                f.mx[a, b] += w * Xa * Yb * nxds
                                f.my[a, b] += w * Xa * Yb * nyds
            else:
                _, sa, sb = item
                for e0, e1, edge in _split_perimeter(sa, sb):
                    length = e1 - e0
                    edge_len[edge] += length
                    # centred coordinates of the segment ends
                    if edge == 0:
                        P0, P1 = (e0 - 0.5, -0.5), (e1 - 0.5, -0.5)
                    elif edge == 1:
                        P0, P1 = (0.5, e0 - 0.5), (0.5, e1 - 0.5)
                    elif edge == 2:
                        P0, P1 = (0.5 - e0, 0.5), (0.5 - e1, 0.5)
                    else:
                        P0, P1 = (-0.5, 0.5 - e0), (-0.5, 0.5 - e1)
                    if edge in (1, 3):
                        Xe = P0[0]
                        for a in range(DEG + 1):
                            for b in range(DEG + 1 - a):
                                mom[a, b] += Xe ** (a + 1) / (a + 1) * (P1[1] ** (b + 1) - P0[1] ** (b + 1)) / (b + 1)
                    if self.box is not None and self._on_border(i, j, edge):
                        f = faces.setdefault(self.box.index, Face(self.box.index))
                        nrm = [(0.0, -1.0), (1.0, 0.0), (0.0, 1.0), (-1.0, 0.0)][edge]
                        _segment_moments(f, P0, P1, nrm)
        return Component(idx, mom, edge_len, faces, loop)

    def _on_border(self, i, j, edge):
        return ((edge == 0 and j == 0) or (edge == 1 and i == self.nx - 1)
                or (edge == 2 and j == self.ny - 1) or (edge == 3 and i == 0))

    def pure_component(self, idx):
        """The full square as a component (exact edge integrals, box faces)."""
        return self._component(idx, [("perim", 0.0, 4.0)])

    def _classify_native(self):
        nx, ny, h = self.nx, self.ny, self.h
        self.native = np.zeros(nx * ny, dtype=np.int8)   # 0 empty, 1 pure, 2 cut
        self.native_comps = {}
        # cell centres: inside test, vectorised per curve
        xs = self.x0 + (np.arange(nx) + 0.5) * h
        ys = self.y0 + (np.arange(ny) + 0.5) * h
        X, Y = np.meshgrid(xs, ys)
        inside = _domain_mask(self.curves, X, Y)
        self.native[:] = np.where(inside.ravel(), 1, 0)
        for idx in sorted(self.cell_arcs):
            self.native[idx] = 2
            loops = self._loops(idx)
            comps = []
            for loop in loops:
                comps.append(self._component(idx, loop))
            for comp in comps:
                if comp.volume <= 0.0:
                    raise GeometryError("non-positive component volume in cell %d" % idx)
            self.native_comps[idx] = comps

    # -- Alg. 1 ------------------------------------------------------------
    def _neighbours(self, idx):
        """Edge neighbours in the order -x, +x, -y, +y with the edge of idx they share."""
        i, j = idx % self.nx, idx // self.nx
        out = []
        if i > 0:
            out.append((idx - 1, 3))
        if i < self.nx - 1:
            out.append((idx + 1, 1))
        if j > 0:
            out.append((idx - self.nx, 0))
        if j < self.ny - 1:
            out.append((idx + self.nx, 2))
        return out

    def aperture(self, idx, edge):
        """Length (units of h) of the cell edge that lies in the domain."""
        k = self.native[idx]
        if k == 0:
            return 0.0
        if k == 1:
            return 1.0
        return sum(c.edge_len[edge] for c in self.native_comps[idx])

    def _merge(self):
        n = self.nx * self.ny
        vol = np.where(self.native == 1, 1.0, 0.0)
        members = {}
        for idx, comps in self.native_comps.items():
            keep = max(range(len(comps)), key=lambda k: (comps[k].volume, -k))
            members.setdefault(idx, []).append((idx, comps[keep]))
            for k, comp in enumerate(comps):
                if k == keep:
                    continue
                best, bl = None, -1.0
                for nb, edge in self._neighbours(idx):
                    if comp.edge_len[edge] > bl + MERGE_TIE:
                        best, bl = nb, comp.edge_len[edge]
                if best is None or bl <= 0.0:
                    raise GeometryError("isolated component in cell %d" % idx)
                members.setdefault(best, []).append((idx, comp))
        for idx in range(n):
            if self.native[idx] == 1 and idx in members:
                members[idx].insert(0, (idx, self.pure_component(idx)))
        for idx, lst in members.items():
            vol[idx] = sum(c.volume for _, c in lst)
        host = np.full(n, -1, dtype=np.int64)
        for idx in range(n):
            if vol[idx] <= 0.0 or vol[idx] > self.theta:
                continue
            if self.native[idx] == 1 and idx not in members:
                continue
            best, bl = None, 0.0
            for nb, edge in self._neighbours(idx):
                if vol[nb] <= 0.0:
                    continue
                ap = self.aperture(idx, edge)
                if ap > bl + MERGE_TIE:   # a tie keeps the earlier neighbour in -x, +x, -y, +y
                    best, bl = nb, ap
            if best is None:
                raise GeometryError("small cell %d has no neighbour to merge into" % idx)
            if best not in members:
                members[best] = [(best, self.pure_component(best))]
            members[best].extend(members.pop(idx, []))
            vol[best] += vol[idx]
            vol[idx] = 0.0
            host[idx] = best
            host[host == idx] = best
        self.vol = vol
        self.host = host
        state = np.full(n, EMPTY, dtype=np.int8)
        state[(self.native != 0) & (vol == 0.0)] = MERGED
        state[vol > 0.0] = CUT
        pure = (self.native == 1) & (vol > 0.0)
        for idx in members:
            pure[idx] = False
        state[pure] = PURE
        self.state = state
        self.cv = {}
        for idx, lst in members.items():
            if vol[idx] <= 0.0:
                continue
            mom = np.zeros((DEG + 1, DEG + 1))
            faces = {}
            i, j = idx % self.nx, idx // self.nx
            for own, comp in lst:
                d = own % self.nx - i
                e = own // self.nx - j
                mom += shift_moments(comp.mom, d, e)
                for cidx, f in comp.faces.items():
                    g = faces.setdefault(cidx, Face(cidx))
                    g.length += f.length
                    g.m += shift_moments(f.m, d, e)
                    g.mx += shift_moments(f.mx, d, e)
                    g.my += shift_moments(f.my, d, e)
            self.cv[idx] = ControlVolume(idx, lst, mom, faces)
        # pure cells on the box border own their border edges as boundary pieces
        self._pure_faces = {}

    # -- queries -------------------------------------------------------------
    def moments(self, idx):
        """Area moments about the cell's own centre (scaled)."""
        if self.state[idx] == PURE:
            return _SQUARE
        return self.cv[idx].mom

    def faces(self, idx):
        """Boundary faces (curve index -> Face) of a non-empty cell, moments
        about the cell's own centre."""
        if self.state[idx] == PURE:
            i, j = idx % self.nx, idx // self.nx
            if self.box is None or not (i == 0 or j == 0 or i == self.nx - 1 or j == self.ny - 1):
                return {}
            if idx not in self._pure_faces:
                self._pure_faces[idx] = self.pure_component(idx).faces
            return self._pure_faces[idx]
        return self.cv[idx].faces

    def volume(self, idx):
        return float(self.vol[idx])

    def total_volume(self):
        return float(self.vol.sum()) * self.h * self.h

    def final_host(self, idx):
        return int(self.host[idx])


_SQUARE = square_moments()


def _split_perimeter(sa, sb):
    """Split the ccw perimeter path [sa, sb] (sb may exceed 4) into per-edge
    pieces (e0, e1, edge) with edge-local coordinates in [0, 1]."""
    out = []
    s = sa
    while s < sb:
        edge_start = math.floor(s)
        nxt = min(sb, edge_start + 1.0)
        e0 = s - edge_start
        e1 = nxt - edge_start
        if e1 > e0:
            out.append((max(0.0, e0), min(1.0, e1), int(edge_start) % 4))
        s = nxt
    return out


def _segment_moments(f, P0, P1, nrm):
    """Exact moments of the straight segment P0->P1 (axis aligned)."""
    L = math.hypot(P1[0] - P0[0], P1[1] - P0[1])
    if L <= 0.0:
        return
    f.length += L
    horizontal = P0[1] == P1[1]
    for a in range(DEG + 1):
        for b in range(DEG + 1 - a):
            if horizontal:
                x0, x1 = sorted((P0[0], P1[0]))
                v = (x1 ** (a + 1) - x0 ** (a + 1)) / (a + 1) * P0[1] ** b
            else:
                y0, y1 = sorted((P0[1], P1[1]))
                v = P0[0] ** a * (y1 ** (b + 1) - y0 ** (b + 1)) / (b + 1)
            f.m[a, b] += v
            f.mx[a, b] += v * nrm[0]
            f.my[a, b] += v * nrm[1]


def _domain_mask(curves, X, Y):
    """Vectorised open-domain membership of points (box handled by the grid)."""
    mask = np.ones(X.shape, dtype=bool)
    for c in curves:
        if c.kind == BOX:
            continue
        if c.kind == CIRCLE:
            cx, cy, r = c.p
            ins = (X - cx) ** 2 + (Y - cy) ** 2 < r * r
        elif c.kind == ELLIPSE:
            cx, cy, a1, a2, rot = c.p
            cr, sr = math.cos(rot), math.sin(rot)
            dx, dy = X - cx, Y - cy
            u = cr * dx + sr * dy
            v = -sr * dx + cr * dy
            ins = (u / a1) ** 2 + (v / a2) ** 2 < 1.0
        elif c.kind == POLYGON:
            v = c.p
            ins = np.ones(X.shape, dtype=bool)
            for k in range(4):
                ax, ay, bx, by = v[2 * k], v[2 * k + 1], v[(2 * k + 2) % 8], v[(2 * k + 3) % 8]
                ins &= (bx - ax) * (Y - ay) - (by - ay) * (X - ax) > 0.0
        else:
            cx, cy, r0, A, k, ph = c.p
            dx, dy = X - cx, Y - cy
            rho = np.hypot(dx, dy)
            th = np.arctan2(dy, dx)
            rr = r0 + A * (np.sin(k * th + ph) if c.kind == POLAR_SIN else np.cos(k * th + ph))
            ins = rho < rr
        mask &= ins if c.inside else ~ins
    return mask


def build_cut_grid(grid, curves, theta=0.3, q=GL_Q):
    return CutGrid(grid, curves, theta=theta, q=q)


# ---------------------------------------------------------------------------
# Cubature of functions over cut cells and boundary faces (Section 2.4)
# ---------------------------------------------------------------------------
def cell_averages(cg, fn, q_pure=6, q=GL_Q):
    """Cell averages <fn>_i on every non-empty cell (grid-shaped array).

    Pure cells: tensor Gauss-Legendre (q_pure^2 nodes).  Cut cells: Green's
    formula with the x-primitive F(x,y) = int_{xi0}^x fn(xi,y) dxi evaluated by
    an inner Gauss-Legendre rule, xi0 = the member cell's centre (eq.
    iteratedIntegral).  Merged cells average over the union."""
    nx, ny, h = cg.nx, cg.ny, cg.h
    out = np.zeros(nx * ny)
    tq, wq = gauss_legendre(q_pure)
    w2 = 0.25 * wq[:, None] * wq[None, :]
    xs = cg.x0 + (np.arange(nx)[None, :, None, None] + 0.5 + 0.5 * tq[None, None, :, None]) * h
    pure_avg = np.zeros((ny, nx))
    rows = max(1, (1 << 22) // (nx * q_pure * q_pure))
    for j0 in range(0, ny, rows):
        j1 = min(ny, j0 + rows)
        ys = cg.y0 + (np.arange(j0, j1)[:, None, None, None] + 0.5 + 0.5 * tq[None, None, None, :]) * h
        vals = fn(xs, ys)
        pure_avg[j0:j1] = (vals * w2[None, None]).sum(axis=(2, 3))
    pure_avg = pure_avg.ravel()
    is_pure = cg.state == PURE
    out[is_pure] = pure_avg[is_pure]
    for idx, cv in cg.cv.items():
        total = 0.0
        for own, comp in cv.members:
            if cg.native[own] == 1:
                total += pure_avg[own]
            else:
                total += _component_integral(cg, own, comp, fn, q)
        out[idx] = total / cv.volume
    return out.reshape(ny, nx)


def _component_integral(cg, own, comp, fn, q):
    """iint over the native component ``comp`` of cell ``own`` of fn, / h^2."""
    return _loop_integral(cg, own, comp.loop, fn, q)


def _loop_integral(cg, own, loop, fn, q):
    h = cg.h
    i, j = own % cg.nx, own // cg.nx
    cx, cy = cg.x0 + (i + 0.5) * h, cg.y0 + (j + 0.5) * h
    tq, wq = gauss_legendre(q)
    total = 0.0

    def prim(x, y):
        # int_{cx}^{x} fn(xi, y) dxi by Gauss-Legendre
        half = 0.5 * (x - cx)
        xi = cx + half * (1.0 + tq)
        return half * float(np.sum(wq * fn(xi, y + 0.0 * xi)))

    for item in loop:
        if item[0] == "arc":
            arc = item[1]
            c = cg.curves[arc.curve]
            for ta, tb in arc.pieces:
                half = 0.5 * (tb - ta)
                mid = 0.5 * (ta + tb)
                for qn in range(q):
                    t = mid + half * tq[qn]
                    px, py = c.point(t)
                    dy = c.deriv(t)[1] * arc.sigma
                    total += wq[qn] * half * prim(px, py) * dy
        else:
            _, sa, sb = item
            for e0, e1, edge in _split_perimeter(sa, sb):
                if edge == 1:
                    xe, ya, yb = cx + 0.5 * h, cy + (e0 - 0.5) * h, cy + (e1 - 0.5) * h
                elif edge == 3:
                    xe, ya, yb = cx - 0.5 * h, cy + (0.5 - e0) * h, cy + (0.5 - e1) * h
                else:
                    continue
                half = 0.5 * (yb - ya)
                for qn in range(q):
                    y = 0.5 * (ya + yb) + half * tq[qn]
                    total += wq[qn] * half * prim(xe, y)
    return total / (h * h)


def face_averages(cg, idx, fn_value, fn_normal=None, q=GL_Q):
    """Boundary-face averages on cell ``idx``: for each curve c touching the
    (merged) cell, <<g>> = int_S g ds / |S| with g = fn_value(x, y) for
    Dirichlet curves or fn_normal(x, y, nx, ny) for Neumann curves."""
    out = {}
    h = cg.h
    tq, wq = gauss_legendre(q)
    mem = cg.cv[idx].members if idx in cg.cv else [(idx, None)]
    acc = {}
    for own, comp in mem:
        i, j = own % cg.nx, own // cg.nx
        cx, cy = cg.x0 + (i + 0.5) * h, cg.y0 + (j + 0.5) * h
        if comp is None or comp.loop is None:
            loops = [[("perim", 0.0, 4.0)]]
        else:
            loops = [comp.loop]
        for loop in loops:
            for item in loop:
                if item[0] == "arc":
                    arc = item[1]
                    c = cg.curves[arc.curve]
                    for ta, tb in arc.pieces:
                        half = 0.5 * (tb - ta)
                        mid = 0.5 * (ta + tb)
                        for qn in range(q):
                            t = mid + half * tq[qn]
                            px, py = c.point(t)
                            dx, dy = c.deriv(t)
                            sp = math.hypot(dx, dy)
                            nxv, nyv = arc.sigma * dy / sp, -arc.sigma * dx / sp
                            g = c.datum(fn_value, fn_normal, px, py, nxv, nyv)
                            w = wq[qn] * half * sp
                            s = acc.setdefault(arc.curve, [0.0, 0.0])
                            s[0] += w * g
                            s[1] += w
                elif cg.box is not None:
                    _, sa, sb = item
                    for e0, e1, edge in _split_perimeter(sa, sb):
                        if not cg._on_border(i, j, edge):
                            continue
                        nrm = [(0.0, -1.0), (1.0, 0.0), (0.0, 1.0), (-1.0, 0.0)][edge]
                        if edge == 0:
                            A, B = (cx + (e0 - 0.5) * h, cy - 0.5 * h), (cx + (e1 - 0.5) * h, cy - 0.5 * h)
                        elif edge == 1:
                            A, B = (cx + 0.5 * h, cy + (e0 - 0.5) * h), (cx + 0.5 * h, cy + (e1 - 0.5) * h)
                        elif edge == 2:
                            A, B = (cx + (0.5 - e0) * h, cy + 0.5 * h), (cx + (0.5 - e1) * h, cy + 0.5 * h)
                        else:
                            A, B = (cx - 0.5 * h, cy + (0.5 - e0) * h), (cx - 0.5 * h, cy + (0.5 - e1) * h)
                        L = math.hypot(B[0] - A[0], B[1] - A[1])
                        for qn in range(q):
                            tt = 0.5 * (1.0 + tq[qn])
                            px, py = A[0] + tt * (B[0] - A[0]), A[1] + tt * (B[1] - A[1])
                            g = cg.box.datum(fn_value, fn_normal, px, py, nrm[0], nrm[1])
                            w = 0.5 * wq[qn] * L
                            s = acc.setdefault(cg.box.index, [0.0, 0.0])
                            s[0] += w * g
                            s[1] += w
    for cidx, (num, den) in acc.items():
        out[cidx] = num / den
    return out
