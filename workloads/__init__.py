"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds *no* arithmetic of the cut-cell method: it only describes
problems (domains as analytic curves, coefficients, manufactured solutions
with their closed-form derivatives) and draws seeded random numbers.  Cell
and boundary averages of these functions are computed by each side with its
own cubature.

Curve descriptors are plain dicts::

    {"kind": BOX|CIRCLE|ELLIPSE|POLAR_SIN|POLAR_COS|POLYGON,
     "p": [...], "inside": 1 if the domain lies inside the curve else 0,
     "bc": DIRICHLET|NEUMANN|ROBIN, "robin": (gamma1, gamma2) for ROBIN}

Parameter layouts: circle ``cx, cy, r``; ellipse ``cx, cy, a1, a2, rot``;
polygon: a convex quadrilateral, ``x0, y0, x1, y1, x2, y2, x3, y3``
counter-clockwise;
polar ``cx, cy, r0, A, k, phase`` with ``r(t) = r0 + A sin(k t + phase)``
(or ``cos``); box ``x0, y0, x1, y1`` (the grid extent).

The problem statement these describe is the elliptic equation
``a u_xx + b u_xy + c u_yy = f`` with ``b^2 - 4ac < 0`` (Section 1,
eq. ccEllipticEq) and Dirichlet, Neumann or Robin data (gamma1 u + gamma2
du/dn, the boundary operator of Section 3) on each boundary curve.
"""
from __future__ import annotations

import math

import numpy as np

BOX, CIRCLE, ELLIPSE, POLAR_SIN, POLAR_COS, POLYGON = 0, 1, 2, 3, 4, 5
DIRICHLET, NEUMANN, ROBIN = 0, 1, 2


def robin(curve, gamma1, gamma2):
    """The same curve with the Robin condition gamma1 u + gamma2 du/dn = g."""
    return dict(curve, bc=ROBIN, robin=(float(gamma1), float(gamma2)))


def box(bc=DIRICHLET, x0=0.0, y0=0.0, x1=1.0, y1=1.0):
    return {"kind": BOX, "p": [x0, y0, x1, y1], "inside": 1, "bc": bc}


def circle(cx, cy, r, inside=0, bc=DIRICHLET):
    return {"kind": CIRCLE, "p": [cx, cy, r], "inside": inside, "bc": bc}


def ellipse(cx, cy, a1, a2, rot=0.0, inside=0, bc=DIRICHLET):
    return {"kind": ELLIPSE, "p": [cx, cy, a1, a2, rot], "inside": inside, "bc": bc}


def polygon(vertices, inside=1, bc=DIRICHLET):
    """Convex quadrilateral with counter-clockwise vertices [(x, y)] * 4."""
    return {"kind": POLYGON, "p": [float(c) for v in vertices for c in v], "inside": inside, "bc": bc}


def rotated_box(theta, cx=0.5, cy=0.5, half=0.5, inside=1, bc=DIRICHLET):
    """The square of side 2 half centred at (cx, cy), rotated
    counter-clockwise by theta about its centre."""
    c, s = math.cos(theta), math.sin(theta)
    corners = [(-half, -half), (half, -half), (half, half), (-half, half)]
    return polygon([(cx + c * x - s * y, cy + s * x + c * y) for x, y in corners], inside, bc)


def rotated(sol, theta, cx=0.5, cy=0.5):
    """u(x) = sol(R(-theta)(x - c) + c): the solution carried along with a
    domain rotated counter-clockwise by theta about c (chain rule for the
    derivatives)."""
    c, s = math.cos(theta), math.sin(theta)

    def xi(x, y):
        dx, dy = x - cx, y - cy
        return cx + c * dx + s * dy, cy - s * dx + c * dy

    def ux(x, y):
        a, b = xi(x, y)
        return c * sol.ux(a, b) - s * sol.uy(a, b)

    def uy(x, y):
        a, b = xi(x, y)
        return s * sol.ux(a, b) + c * sol.uy(a, b)

    def uxx(x, y):
        a, b = xi(x, y)
        return c * c * sol.uxx(a, b) - 2 * c * s * sol.uxy(a, b) + s * s * sol.uyy(a, b)

    def uyy(x, y):
        a, b = xi(x, y)
        return s * s * sol.uxx(a, b) + 2 * c * s * sol.uxy(a, b) + c * c * sol.uyy(a, b)

    def uxy(x, y):
        a, b = xi(x, y)
        return c * s * sol.uxx(a, b) + (c * c - s * s) * sol.uxy(a, b) - c * s * sol.uyy(a, b)

    return Manufactured("%s rotated by %.6f" % (sol.name, theta), lambda x, y: sol.u(*xi(x, y)), ux, uy, uxx, uxy,
                        uyy)


def polar_sin(cx, cy, r0, A, k, phase=0.0, inside=0, bc=DIRICHLET):
    return {"kind": POLAR_SIN, "p": [cx, cy, r0, A, float(k), phase], "inside": inside, "bc": bc}


def polar_cos(cx, cy, r0, A, k, phase=0.0, inside=0, bc=DIRICHLET):
    return {"kind": POLAR_COS, "p": [cx, cy, r0, A, float(k), phase], "inside": inside, "bc": bc}


# ---------------------------------------------------------------------------
# Manufactured solutions: value, gradient and second derivatives in closed form.
# ---------------------------------------------------------------------------
class Manufactured:
    """u and its derivatives; ``f`` applies a u_xx + b u_xy + c u_yy."""

    def __init__(self, name, u, ux, uy, uxx, uxy, uyy):
        self.name = name
        self.u, self.ux, self.uy = u, ux, uy
        self.uxx, self.uxy, self.uyy = uxx, uxy, uyy

    def f(self, a, b, c):
        return lambda x, y: a * self.uxx(x, y) + b * self.uxy(x, y) + c * self.uyy(x, y)

    def dudn(self, x, y, nx, ny):
        return self.ux(x, y) * nx + self.uy(x, y) * ny

    def datum(self, curve, x, y, nx, ny):
        """The boundary datum of a curve descriptor at points with outward
        normals n: u, du/dn or gamma1 u + gamma2 du/dn."""
        if curve["bc"] == DIRICHLET:
            return self.u(x, y)
        if curve["bc"] == NEUMANN:
            return self.dudn(x, y, nx, ny)
        g1, g2 = curve["robin"]
        return g1 * self.u(x, y) + g2 * self.dudn(x, y, nx, ny)


PI = math.pi

SIN2PIX_EXPY = Manufactured(
    "sin(2 pi x) exp(y)",
    lambda x, y: np.sin(2 * PI * x) * np.exp(y),
    lambda x, y: 2 * PI * np.cos(2 * PI * x) * np.exp(y),
    lambda x, y: np.sin(2 * PI * x) * np.exp(y),
    lambda x, y: -4 * PI * PI * np.sin(2 * PI * x) * np.exp(y),
    lambda x, y: 2 * PI * np.cos(2 * PI * x) * np.exp(y),
    lambda x, y: np.sin(2 * PI * x) * np.exp(y),
)

EXPX_COS3Y = Manufactured(
    "exp(x) cos(3y)",
    lambda x, y: np.exp(x) * np.cos(3 * y),
    lambda x, y: np.exp(x) * np.cos(3 * y),
    lambda x, y: -3 * np.exp(x) * np.sin(3 * y),
    lambda x, y: np.exp(x) * np.cos(3 * y),
    lambda x, y: -3 * np.exp(x) * np.sin(3 * y),
    lambda x, y: -9 * np.exp(x) * np.cos(3 * y),
)

SINPIX_SINPIY = Manufactured(
    "sin(pi x) sin(pi y)",
    lambda x, y: np.sin(PI * x) * np.sin(PI * y),
    lambda x, y: PI * np.cos(PI * x) * np.sin(PI * y),
    lambda x, y: PI * np.sin(PI * x) * np.cos(PI * y),
    lambda x, y: -PI * PI * np.sin(PI * x) * np.sin(PI * y),
    lambda x, y: PI * PI * np.cos(PI * x) * np.cos(PI * y),
    lambda x, y: -PI * PI * np.sin(PI * x) * np.sin(PI * y),
)

SIN4X_COS3Y = Manufactured(
    "sin(4x) cos(3y)",
    lambda x, y: np.sin(4 * x) * np.cos(3 * y),
    lambda x, y: 4 * np.cos(4 * x) * np.cos(3 * y),
    lambda x, y: -3 * np.sin(4 * x) * np.sin(3 * y),
    lambda x, y: -16 * np.sin(4 * x) * np.cos(3 * y),
    lambda x, y: -12 * np.cos(4 * x) * np.sin(3 * y),
    lambda x, y: -9 * np.sin(4 * x) * np.cos(3 * y),
)

SINPIX_SIN2PIY_X3 = Manufactured(
    "sin(pi x) sin(2 pi y) + x^3",
    lambda x, y: np.sin(PI * x) * np.sin(2 * PI * y) + x ** 3,
    lambda x, y: PI * np.cos(PI * x) * np.sin(2 * PI * y) + 3 * x ** 2,
    lambda x, y: 2 * PI * np.sin(PI * x) * np.cos(2 * PI * y) + 0 * x,
    lambda x, y: -PI * PI * np.sin(PI * x) * np.sin(2 * PI * y) + 6 * x,
    lambda x, y: 2 * PI * PI * np.cos(PI * x) * np.cos(2 * PI * y),
    lambda x, y: -4 * PI * PI * np.sin(PI * x) * np.sin(2 * PI * y) + 0 * x,
)


def polynomial(coeffs):
    """Manufactured polynomial sum_{(p,q)} c x^p y^q given as {(p, q): c}."""
    def term(dp, dq):
        def fn(x, y):
            out = 0.0 * x + 0.0 * y
            for (p, q), c in coeffs.items():
                if p < dp or q < dq:
                    continue
                k = c
                for s in range(dp):
                    k *= (p - s)
                for s in range(dq):
                    k *= (q - s)
                out = out + k * x ** (p - dp) * y ** (q - dq)
            return out
        return fn
    return Manufactured("poly", term(0, 0), term(1, 0), term(0, 1), term(2, 0), term(1, 1), term(0, 2))


def fourier_rhs(seed, modes=8):
    """f = sum_{p,q<=modes} c_pq sin(p pi x) sin(q pi y), c_pq ~ N(0,1)."""
    c = np.random.default_rng(seed).standard_normal((modes, modes))

    def f(x, y):
        out = 0.0 * x
        for p in range(modes):
            sx = np.sin((p + 1) * PI * x)
            for q in range(modes):
                out = out + c[p, q] * sx * np.sin((q + 1) * PI * y)
        return out
    return f, c


# ---------------------------------------------------------------------------
# Seeded geometries.
# ---------------------------------------------------------------------------
def random_circles(seed, count, rmin, rmax, clearance=0.05, lo=0.0, hi=1.0):
    """Non-overlapping circles in the box [lo,hi]^2, drawn by rejection."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        r = rng.uniform(rmin, rmax)
        cx = rng.uniform(lo + r + clearance, hi - r - clearance)
        cy = rng.uniform(lo + r + clearance, hi - r - clearance)
        if all(math.hypot(cx - q[0], cy - q[1]) >= r + q[2] + clearance for q in out):
            out.append((cx, cy, r))
    return [circle(cx, cy, r) for cx, cy, r in out]


def random_ellipses(seed, count, amin, amax, clearance=0.05, lo=0.0, hi=1.0, bc=DIRICHLET):
    """Non-overlapping ellipses (bounding circles kept apart), random rotation."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        a1, a2 = rng.uniform(amin, amax, size=2)
        rot = rng.uniform(0.0, PI)
        R = max(a1, a2)
        cx = rng.uniform(lo + R + clearance, hi - R - clearance)
        cy = rng.uniform(lo + R + clearance, hi - R - clearance)
        if all(math.hypot(cx - q[0], cy - q[1]) >= R + q[2] + clearance for q in out):
            out.append((cx, cy, R, a1, a2, rot))
    return [ellipse(cx, cy, a1, a2, rot, bc=bc) for cx, cy, R, a1, a2, rot in out]


def _r4cos3t():
    """u = r^4 cos 3t = r p with p = x^3 - 3 x y^2 (Problem 1 of Section 5.1);
    derivatives by the product rule with r_x = x/r, r_xx = y^2/r^3,
    r_xy = -x y/r^3, r_yy = x^2/r^3."""
    def r(x, y):
        return np.sqrt(x * x + y * y)

    def p(x, y):
        return x ** 3 - 3 * x * y * y

    def ux(x, y):
        rr = r(x, y)
        return x / rr * p(x, y) + rr * (3 * x * x - 3 * y * y)

    def uy(x, y):
        rr = r(x, y)
        return y / rr * p(x, y) + rr * (-6 * x * y)

    def uxx(x, y):
        rr = r(x, y)
        return y * y / rr ** 3 * p(x, y) + 2 * x / rr * (3 * x * x - 3 * y * y) + rr * 6 * x

    def uyy(x, y):
        rr = r(x, y)
        return x * x / rr ** 3 * p(x, y) + 2 * y / rr * (-6 * x * y) + rr * (-6 * x)

    def uxy(x, y):
        rr = r(x, y)
        return (-x * y / rr ** 3 * p(x, y) + x / rr * (-6 * x * y) + y / rr * (3 * x * x - 3 * y * y)
                + rr * (-6 * y))

    return Manufactured("r^4 cos(3 theta)", lambda x, y: r(x, y) * p(x, y), ux, uy, uxx, uxy, uyy)


R4COS3T = _r4cos3t()


def grid(n, x0=0.0, y0=0.0, length=1.0):
    return {"x0": x0, "y0": y0, "h": length / n, "nx": n, "ny": n}


def config(k, n=None):
    """The five synthetic workloads.  Returns a dict with grid, curves, (a,b,c),
    manufactured solution (or None) and the right-hand side function."""
    if k == 1:
        n = n or 64
        curves = [circle(0.5, 0.5, 0.3, inside=1)]
        a, b, c = 1.0, 0.0, 1.0
        sol = SIN2PIX_EXPY
    elif k == 2:
        n = n or 1024
        curves = [box(), polar_sin(0.5, 0.5, 0.25, 0.05, 5, bc=NEUMANN)]
        a, b, c = 1.0, 0.5, 1.0
        sol = EXPX_COS3Y
    elif k == 3:
        n = n or 512
        curves = [box(), circle(0.5, 0.5, 0.2)]
        a, b, c = 1.0, 0.0, 1.0
        sol = None
    elif k == 4:
        n = n or 2048
        curves = [box()] + random_circles(4, 3, 0.05, 0.15)
        a, b, c = 1.0, 0.0, 1.0
        sol = SINPIX_SINPIY
    elif k == 5:
        n = n or 4096
        curves = [box()] + random_ellipses(5, 5, 0.03, 0.12)
        a, b, c = 1.0, 1.2, 1.0
        sol = SINPIX_SIN2PIY_X3
    else:
        raise ValueError(k)
    out = {"id": k, "grid": grid(n), "curves": curves, "a": a, "b": b, "c": c, "solution": sol}
    if sol is not None:
        out["f"] = sol.f(a, b, c)
    else:
        out["f"] = fourier_rhs(3000)[0]
    return out


def batch_geometries(count=32, seed0=3100):
    """Config-3 geometry batch: grid sizes from {128,...,1024}, 1-3 ellipses."""
    out = []
    for g in range(count):
        rng = np.random.default_rng(seed0 + g)
        n = int(rng.choice([128, 256, 512, 1024]))
        m = int(rng.integers(1, 4))
        curves = [box()] + random_ellipses(seed0 + 1000 + g, m, 0.05, 0.2)
        out.append({"id": f"3g{g}", "grid": grid(n), "curves": curves, "a": 1.0, "b": 0.0, "c": 1.0,
                    "solution": None, "f": fourier_rhs(3000 + g)[0]})
    return out


def problem2(n, hole_bc=NEUMANN):
    """Poisson on [0,1]^2 minus the ellipse c=(1/2,1/2), a=(1/8,1/4) (Section 5.1, Problem 2)."""
    return {"id": "P2", "grid": grid(n), "curves": [box(), ellipse(0.5, 0.5, 0.125, 0.25, 0.0, bc=hole_bc)],
            "a": 1.0, "b": 0.0, "c": 1.0, "solution": SINPIX_SINPIY, "f": SINPIX_SINPIY.f(1.0, 0.0, 1.0)}


def problem3(n):
    """(a, b, c) = (1, 0, 2) on the unit box, Dirichlet, u = sin(4x) cos(3y)
    (Section 5.1, Problem 3, case (i))."""
    return {"id": "P3", "grid": grid(n), "curves": [box()], "a": 1.0, "b": 0.0, "c": 2.0,
            "solution": SIN4X_COS3Y, "f": SIN4X_COS3Y.f(1.0, 0.0, 2.0)}


def problem2_robin(n, gamma1=1.0, gamma2=0.5):
    """Problem 2's domain and solution with the Robin condition
    gamma1 u + gamma2 du/dn = g on the ellipse (Dirichlet on the box)."""
    cfg = problem2(n, DIRICHLET)
    cfg["id"] = "P2R"
    cfg["curves"] = [cfg["curves"][0], robin(cfg["curves"][1], gamma1, gamma2)]
    return cfg


def problem3_rotated(n):
    """Problem 3 case (ii) (Section 5.1): the unit box rotated counter-clockwise
    by pi/6 about its centre, (a, b, c) = (5/4, -sqrt(3)/2, 7/4) (case (i)'s
    operator in the rotated frame), Dirichlet, u = sin(4x) cos(3y) rotated
    with the domain.  ``n`` is 1/h; the grid covers [-1/4, 5/4]^2 (3n/2 cells
    a side), which holds the rotated box."""
    th = math.pi / 6
    sol = rotated(SIN4X_COS3Y, th)
    a, b, c = 1.25, -math.sqrt(3.0) / 2.0, 1.75
    m = (3 * n) // 2
    return {"id": "P3R", "grid": grid(m, -0.25, -0.25, 1.5), "curves": [rotated_box(th)], "a": a, "b": b, "c": c,
            "solution": sol, "f": sol.f(a, b, c)}


def problem(name, n):
    """The paper's test problems by name: P1, P2N (Neumann on the ellipse),
    P2D (Dirichlet on it), P2R (Robin on it), P3 (case (i)), P3R (case (ii),
    ``n`` = 1/h)."""
    return {"P1": lambda: problem1(n), "P2N": lambda: problem2(n, NEUMANN), "P2D": lambda: problem2(n, DIRICHLET),
            "P2R": lambda: problem2_robin(n), "P3": lambda: problem3(n), "P3R": lambda: problem3_rotated(n)}[name]()


def problem1(n):
    """Poisson on the box [-1/2, 1/2]^2 minus the flower r >= 0.25 + 0.05 cos 6t
    (Section 5.1, Problem 1): Dirichlet on the box, Neumann on the flower,
    u = r^4 cos 3t."""
    return {"id": "P1", "grid": grid(n, -0.5, -0.5), "curves": [box(x0=-0.5, y0=-0.5, x1=0.5, y1=0.5),
                                                            polar_cos(0.0, 0.0, 0.25, 0.05, 6, bc=NEUMANN)],
            "a": 1.0, "b": 0.0, "c": 1.0, "solution": R4COS3T, "f": R4COS3T.f(1.0, 0.0, 1.0)}


def random_field(seed, shape):
    return np.random.default_rng(seed).standard_normal(shape)
