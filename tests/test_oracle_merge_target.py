"""Pins of Alg. 1's merge target (Section 3.1): a small cut cell merges into
the non-empty edge neighbour with which it shares the longest cut face,
ties broken in the order -x, +x, -y, +y.

The domains are convex quadrilaterals, so every cut cell is the grid square
clipped by four half-planes.  Volumes and cut-face lengths are computed here
in closed form (polygon clipping of the square, segment clipping of its
edges), independently of the oracle's Green's-formula cubature and its
boundary tracing.  The expected host of each small cell follows from those
numbers alone; the test checks the cells whose four neighbours are all
either empty or large (no other small cell takes part in their merge).

* The diamond (edges of slope +-1 through half-offset points) cuts corner
  triangles whose two legs are equal: every small cell is a tie, between
  -x and -y, +x and +y, +x and -y, or -x and +y, depending on the edge.
* The rotated rectangle (edges at about 34 and 124 degrees) cuts small
  cells whose longest and shortest cut faces differ: the longest must win.
"""
import numpy as np
import pytest

import workloads as W
from oracle.geometry import build_cut_grid

THETA = 0.3


def _halfplanes(verts):
    """Counter-clockwise vertices -> (point, direction) of each edge; the
    domain lies to the left of every edge."""
    return [(verts[k], (verts[(k + 1) % 4][0] - verts[k][0], verts[(k + 1) % 4][1] - verts[k][1]))
            for k in range(4)]


def _side(hp, x, y):
    (x0, y0), (dx, dy) = hp
    return dx * (y - y0) - dy * (x - x0)


def _clip_polygon(poly, hps):
    """Sutherland-Hodgman clipping of a convex polygon by half-planes."""
    for hp in hps:
        out = []
        for k in range(len(poly)):
            P, Q = poly[k], poly[(k + 1) % len(poly)]
            sp, sq = _side(hp, *P), _side(hp, *Q)
            if sp >= 0:
                out.append(P)
            if (sp >= 0) != (sq >= 0):
                t = sp / (sp - sq)
                out.append((P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1])))
        poly = out
        if not poly:
            break
    return poly


def _area(poly):
    return 0.5 * abs(sum(poly[k][0] * poly[(k + 1) % len(poly)][1] - poly[(k + 1) % len(poly)][0] * poly[k][1]
                         for k in range(len(poly)))) if len(poly) >= 3 else 0.0


def _clip_length(P, Q, hps):
    """Length of the part of segment PQ inside all half-planes."""
    t0, t1 = 0.0, 1.0
    for hp in hps:
        sp, sq = _side(hp, *P), _side(hp, *Q)
        if sp < 0 and sq < 0:
            return 0.0
        if sp < 0:
            t0 = max(t0, sp / (sp - sq))
        elif sq < 0:
            t1 = min(t1, sp / (sp - sq))
    return max(0.0, t1 - t0) * np.hypot(Q[0] - P[0], Q[1] - P[1])


def _expected(n, verts):
    """Closed-form cut cells of the quadrilateral (vertices in cell units)
    on an n x n grid: volume of every cell (units of h^2) and, for every
    small cell whose neighbours are all empty or large, the neighbour Alg. 1
    must pick with the cut-face lengths of its four edges."""
    hps = _halfplanes(verts)
    vol = np.zeros(n * n)
    for j in range(n):
        for i in range(n):
            vol[j * n + i] = _area(_clip_polygon([(i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)], hps))
    out = {}
    for idx in np.flatnonzero((vol > 0) & (vol <= THETA)):
        i, j = idx % n, idx // n
        # edge neighbours in the order -x, +x, -y, +y, with the shared edge
        nbs = [(idx - 1, ((i, j), (i, j + 1))) if i > 0 else None,
               (idx + 1, ((i + 1, j), (i + 1, j + 1))) if i < n - 1 else None,
               (idx - n, ((i, j), (i + 1, j))) if j > 0 else None,
               (idx + n, ((i, j + 1), (i + 1, j + 1))) if j < n - 1 else None]
        if any(nb is not None and 0 < vol[nb[0]] <= THETA for nb in nbs):
            continue   # another small cell could take part: not a clean case
        best, bl, faces = None, 0.0, []
        for nb in nbs:
            length = _clip_length(*nb[1], hps) if nb is not None else 0.0
            faces.append(length)
            # equal lengths (up to the rounding of this closed form) keep
            # the earlier neighbour
            if nb is not None and vol[nb[0]] > 0 and length > bl + 1e-9:
                best, bl = nb[0], length
        out[int(idx)] = (best, faces)
    return vol, out


def _run(n, verts):
    curve = W.polygon([(x / n, y / n) for x, y in verts], inside=1)
    cg = build_cut_grid(W.grid(n), [curve], theta=THETA)
    vol, exp = _expected(n, verts)
    assert np.max(np.abs(cg.vol.sum() - vol.sum())) < 1e-11
    return cg, vol, exp


def test_merge_target_ties_follow_the_order_minus_x_plus_x_minus_y_plus_y():
    n = 32
    # line constants x + y = 43.6, 20.6 and y - x = 11.65, -11.35 (cell units):
    # corner triangles with legs 0.6, 0.4, 0.65, 0.35, all below theta h^2
    cx, cy, r = 15.975, 16.125, 11.5
    verts = [(cx, cy - r), (cx + r, cy), (cx, cy + r), (cx - r, cy)]
    cg, vol, exp = _run(n, verts)
    ties = {}
    for idx, (best, faces) in exp.items():
        assert cg.host[idx] == best, (idx, faces)
        pos = [k for k in range(4) if faces[k] > 0]
        if len(pos) == 2 and abs(faces[pos[0]] - faces[pos[1]]) < 1e-9:
            ties[tuple(pos)] = ties.get(tuple(pos), 0) + 1
    # all four kinds of corner triangle occur, each an exact tie:
    # (-x,-y) -> -x, (+x,+y) -> +x, (+x,-y) -> +x, (-x,+y) -> -x
    assert set(ties) == {(0, 2), (1, 3), (1, 2), (0, 3)}, ties
    assert all(v >= 5 for v in ties.values()), ties
    # every cell with closed-form volume <= theta h^2 was merged, no other
    small = np.flatnonzero((vol > 0) & (vol <= THETA))
    assert set(np.flatnonzero(cg.host >= 0)) == set(small)


def test_merge_target_is_the_longest_cut_face():
    n = 32
    # a rectangle rotated by about 34 degrees: isolated corner triangles
    # and trapezoids with legs of different lengths on all four edges
    verts = [(13.049, 1.241), (30.932, 13.406), (19.146, 30.733), (1.262, 18.567)]
    cg, vol, exp = _run(n, verts)
    distinct = 0
    for idx, (best, faces) in exp.items():
        assert cg.host[idx] == best, (idx, faces)
        pos = sorted(f for f in faces if f > 0)
        if len(pos) >= 2 and pos[-1] > pos[0] + 0.05:
            distinct += 1
    # slivers along all four edges whose longest face is clearly longer
    # than their shortest non-zero one
    assert distinct >= 20, distinct
    small = np.flatnonzero((vol > 0) & (vol <= THETA))
    assert set(np.flatnonzero(cg.host >= 0)) == set(small)
