"""Contact angle of a static drop from the oracle's density field (Section 3.2).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke
check and the benchmark's CPU-baseline leg are its only users, and it shares
no code with the product's contour kernel or its Python analysis helpers.

The paper measures the angle by fitting a circle to the interface of the
static drop, taken as the iso-line rho^A = 0.5, and taking the angle between
the circle's tangent at the contact line and the plane (Section 3.2).  Written
out plainly here:

1. Interface points: every lattice edge between two fluid nodes (right and up
   neighbours, no wrap) whose ends lie on different sides of the level, i.e.
   (a < L) != (b < L), gives the linearly interpolated point a + t (b - a),
   t = (L - a) / (b - a).  Points of edges with a solid node within chessboard
   distance `skip` of either end are dropped (the interface bends inside the
   diffuse wall layer; the circle describes the drop away from it).
2. Circle: least-squares fit of x^2 + y^2 + D x + E y + F = 0 to the points
   (algebraic fit), solved with numpy's lstsq.
3. Wall: the straight line through the half-way points between the top solid
   node of each column and the fluid node above it (bounce-back places the
   wall half-way), fitted by least squares.
4. Angle: with h the signed distance of the circle centre from the wall
   (positive on the fluid side) and R the radius, cos(theta) = -h / R, theta
   measured through the drop.
"""
from __future__ import annotations

import math

import numpy as np


def interface_points(rhoA, mask, level=0.5, skip=3, roi=None):
    """Interpolated crossings of rho^A = level on fluid-fluid edges (step 1).

    roi = (x0, y0, x1, y1), inclusive; both ends of an edge must lie in it."""
    a = np.asarray(rhoA, dtype=np.float64)
    solid = np.asarray(mask) != 0
    ny, nx = a.shape
    x0, y0, x1, y1 = roi if roi is not None else (0, 0, nx - 1, ny - 1)
    # solid within chessboard distance `skip`: shifted copies, wrapped (borders
    # of a non-periodic box are solid, so wrapping adds nothing new there)
    near = np.zeros_like(solid)
    for dy in range(-skip, skip + 1):
        for dx in range(-skip, skip + 1):
            near |= np.roll(np.roll(solid, dy, axis=0), dx, axis=1)
    pts = []
    for y in range(y0, y1 + 1):
        for x in range(x0, x1 + 1):
            if solid[y, x]:
                continue
            for (xb, yb) in ((x + 1, y), (x, y + 1)):
                if xb > x1 or yb > y1 or solid[yb, xb]:
                    continue
                va, vb = a[y, x], a[yb, xb]
                if (va < level) == (vb < level):
                    continue
                if near[y, x] or near[yb, xb]:
                    continue
                t = (level - va) / (vb - va)
                pts.append((x + t * (xb - x), y + t * (yb - y)))
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


def fit_circle(points):
    """Algebraic least-squares circle (step 2): returns (xc, yc, R)."""
    p = np.asarray(points, dtype=np.float64)
    x, y = p[:, 0], p[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -D / 2.0, -E / 2.0
    return xc, yc, math.sqrt(xc * xc + yc * yc - F)


def radial_residuals(points, circle):
    """Distances of the points from the fitted circle (rms, max)."""
    xc, yc, R = circle
    p = np.asarray(points, dtype=np.float64)
    d = np.hypot(p[:, 0] - xc, p[:, 1] - yc) - R
    return float(np.sqrt(np.mean(d * d))), float(np.max(np.abs(d)))


def wall_line(mask, columns=None):
    """Least-squares line y = a x + b through the half-way wall points (step 3).

    For each column in `columns` (default: every interior column) the first
    fluid node above the bottom border is found and the wall point is half a
    node below it.  Columns with no fluid node, and columns whose first fluid
    node is row 1 (there the bottom border, not the plane, is the wall), are
    skipped."""
    m = np.asarray(mask) != 0
    ny, nx = m.shape
    cols = range(1, nx - 1) if columns is None else columns
    xs, ys = [], []
    for x in cols:
        fluid = np.nonzero(~m[1:, x])[0]
        if fluid.size == 0 or fluid[0] == 0:
            continue
        xs.append(float(x))
        ys.append(float(fluid[0] + 1) - 0.5)
    xs, ys = np.array(xs), np.array(ys)
    a, b = np.polyfit(xs, ys, 1)
    return float(a), float(b)


def angle(circle, line):
    """Contact angle in degrees through the drop (step 4); fluid above the line."""
    xc, yc, R = circle
    a, b = line
    h = (yc - (a * xc + b)) / math.sqrt(1.0 + a * a)
    return math.degrees(math.acos(max(-1.0, min(1.0, -h / R))))


def measure(rhoA, mask, *, level=0.5, skip=3, roi=None, columns=None):
    """Steps 1-4 in order; returns dict(theta, xc, yc, R, n, rms, max_dev)."""
    pts = interface_points(rhoA, mask, level, skip, roi)
    c = fit_circle(pts)
    rms, mx = radial_residuals(pts, c)
    return dict(theta=angle(c, wall_line(mask, columns)), xc=c[0], yc=c[1], R=c[2], n=len(pts),
                rms=rms, max_dev=mx)
