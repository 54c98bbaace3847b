"""Pins of the oracle's cut-cell geometry (Section 3.1, Alg. 1, Section 2.4)
against closed forms that do not use the oracle's own formulas."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.geometry import (CUT, EMPTY, MERGED, PURE, GeometryError, build_cut_grid,
                             cell_averages, gauss_legendre)


def _integral(cg, a, b, cx=0.5, cy=0.5):
    """sum over non-empty cells of int (x-cx)^a (y-cy)^b, rebuilt from the
    scaled moments about each cell centre by the binomial theorem."""
    h = cg.h
    total = 0.0
    for idx in np.flatnonzero(cg.vol > 0):
        i, j = idx % cg.nx, idx // cg.nx
        dx = cg.x0 + (i + 0.5) * h - cx
        dy = cg.y0 + (j + 0.5) * h - cy
        m = cg.moments(idx)
        for p in range(a + 1):
            for q in range(b + 1):
                total += (math.comb(a, p) * math.comb(b, q) * dx ** (a - p) * dy ** (b - q)
                          * h ** (p + q) * m[p, q])
    return total * h * h


@pytest.mark.parametrize("n", [32, 64])
def test_disk_area_perimeter_and_moments(n):
    R = 0.3
    cg = build_cut_grid(W.grid(n), [W.circle(0.5, 0.5, R, inside=1)])
    assert abs(cg.total_volume() - math.pi * R * R) < 1e-14
    length = sum(f.length for cv in cg.cv.values() for f in cv.faces.values()) * cg.h
    assert abs(length - 2 * math.pi * R) < 1e-13
    # int (x-1/2)^2 over the disk = pi R^4 / 4; int (x-1/2)^2 (y-1/2)^2 = pi R^6 / 24
    assert abs(_integral(cg, 2, 0) - math.pi * R ** 4 / 4) < 1e-14
    assert abs(_integral(cg, 0, 2) - math.pi * R ** 4 / 4) < 1e-14
    assert abs(_integral(cg, 2, 2) - math.pi * R ** 6 / 24) < 1e-15
    assert abs(_integral(cg, 1, 0)) < 1e-15 and abs(_integral(cg, 3, 1)) < 1e-15


@pytest.mark.parametrize("n", [48, 96])
def test_rotated_square_area_perimeter_and_moments(n):
    """The unit square rotated by pi/6 about (1/2, 1/2) (a polygon curve,
    the domain of Problem 3 case (ii)) on a grid over [-1/4, 5/4]^2: area 1,
    perimeter 4, centroid (1/2, 1/2), isotropic second moments 1/12 with no
    product term, and the rotation-invariant fourth moment of the square
    (int r^4 dA = 7/180 for the unit square) -- closed forms independent of
    the rotation."""
    cfg = W.problem3_rotated(2 * n // 3)
    cg = build_cut_grid(W.grid(n, -0.25, -0.25, 1.5), cfg["curves"])
    assert abs(cg.total_volume() - 1.0) < 1e-14
    length = sum(f.length for cv in cg.cv.values() for f in cv.faces.values()) * cg.h
    assert abs(length - 4.0) < 1e-13
    assert abs(_integral(cg, 1, 0)) < 1e-15 and abs(_integral(cg, 0, 1)) < 1e-15
    assert abs(_integral(cg, 2, 0) - 1.0 / 12) < 1e-14 and abs(_integral(cg, 0, 2) - 1.0 / 12) < 1e-14
    assert abs(_integral(cg, 1, 1)) < 1e-14
    r4 = _integral(cg, 4, 0) + 2 * _integral(cg, 2, 2) + _integral(cg, 0, 4)
    assert abs(r4 - 7.0 / 180) < 1e-14


def test_box_minus_shapes_areas():
    curves = [W.box(), W.ellipse(0.3, 0.35, 0.12, 0.07, 0.4), W.polar_sin(0.68, 0.62, 0.15, 0.03, 5, 0.3)]
    cg = build_cut_grid(W.grid(64), curves)
    exact = 1.0 - math.pi * 0.12 * 0.07 - math.pi * (0.15 ** 2 + 0.03 ** 2 / 2)
    assert abs(cg.total_volume() - exact) < 1e-14
    cfg = W.config(4, n=64)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    exact = 1.0 - sum(math.pi * c["p"][2] ** 2 for c in cfg["curves"][1:])
    assert abs(cg.total_volume() - exact) < 1e-14


def test_quadrature_order_agreement():
    cfg = W.config(2, n=32)
    a = build_cut_grid(cfg["grid"], cfg["curves"], q=16)
    b = build_cut_grid(cfg["grid"], cfg["curves"], q=32)
    assert np.array_equal(a.state, b.state)
    for idx, cv in a.cv.items():
        assert np.max(np.abs(cv.mom - b.cv[idx].mom)) < 1e-14
    t, w = gauss_legendre(16)
    assert abs(np.sum(w * t ** 30) - 2.0 / 31) < 1e-15     # exact to degree 31


def test_merging_postconditions():
    theta = 0.3
    for k in (1, 2, 4, 5):
        cfg = W.config(k, n=64)
        cg = build_cut_grid(cfg["grid"], cfg["curves"], theta=theta)
        ne = cg.vol > 0
        assert np.all(cg.vol[ne] > theta)              # no small cells remain
        assert np.all(cg.vol[cg.state == PURE] == 1.0)
        assert np.all((cg.host >= 0) == (cg.state == MERGED))
        hosts = cg.host[cg.host >= 0]
        assert np.all(cg.vol[hosts] > 0)               # hosts are live cells
        # merged cells are edge neighbours of some member of their host
        for idx in np.flatnonzero(cg.state == MERGED):
            assert idx in [own for own, _ in cg.cv[cg.host[idx]].members]


def test_pure_box_classification():
    n = 32
    cg = build_cut_grid(W.grid(n), [W.box()])
    assert np.all(cg.state == PURE)
    assert cg.total_volume() == 1.0
    border = [idx for idx in range(n * n) if cg.faces(idx)]
    assert len(border) == 4 * n - 4


def test_disk_kinds_symmetric():
    """A disk centred in the grid: cell states are invariant under the
    symmetries of the square (checks orientation handling of the loops)."""
    cg = build_cut_grid(W.grid(64), [W.circle(0.5, 0.5, 0.3, inside=1)])
    S = cg.state.reshape(64, 64)
    for T in (S[:, ::-1], S[::-1, :], S.T):
        assert np.array_equal(S, T)
    V = cg.vol.reshape(64, 64)
    assert np.max(np.abs(V - V.T)) < 1e-13 and np.max(np.abs(V - V[:, ::-1])) < 1e-13


def test_cell_average_of_polynomial_exact():
    """<x^2 y> over cut cells by the Green's-formula cubature equals the
    moment-based value (two different routes through the geometry)."""
    cfg = W.config(1, n=32)
    cg = build_cut_grid(cfg["grid"], cfg["curves"])
    avg = cell_averages(cg, lambda x, y: x * x * y).ravel()
    h = cg.h
    for idx in np.flatnonzero(cg.vol > 0):
        i, j = idx % cg.nx, idx // cg.nx
        cx, cy = cg.x0 + (i + 0.5) * h, cg.y0 + (j + 0.5) * h
        m = cg.moments(idx)
        v = 0.0
        for p in range(3):
            for q in range(2):
                v += math.comb(2, p) * cx ** (2 - p) * h ** p * math.comb(1, q) * cy ** (1 - q) * h ** q * m[p, q]
        assert abs(v / m[0, 0] - avg[idx]) < 1e-14


def test_rejects_bad_geometry():
    with pytest.raises(GeometryError):
        build_cut_grid(W.grid(32), [W.box(), W.circle(0.95, 0.5, 0.2)])      # leaves the box
    with pytest.raises(GeometryError):
        build_cut_grid(W.grid(32), [W.box(), W.circle(0.515, 0.515, 0.005)])  # inside one cell
    with pytest.raises(GeometryError):
        build_cut_grid(W.grid(32), [W.box(x1=0.9), W.circle(0.5, 0.5, 0.2)])  # box != grid
