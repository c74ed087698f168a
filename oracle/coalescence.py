"""Bridge radius of two coalescing drops from the oracle's density field (Section 4).

TEST INFRASTRUCTURE ONLY, like the rest of this package; shares no code with
the product's line-probe kernel or its analysis helpers.

The paper follows the bridge radius b, the distance between the surface and
the interface of the liquid bridge that joins two sessile drops, and fits
b ~ t^alpha in the viscous regime (alpha = 0.857 expected in 2D).  Written
out plainly here:

1. Crossing along a lattice line: from the start node, step by (dx, dy) and
   take the first node k whose rho^A is below the level.  The crossing lies
   between nodes k - 1 and k at k - 1 + (r_{k-1} - L) / (r_{k-1} - r_k) node
   steps from the start.  If the start node is already below the level the
   crossing is the half-way wall just before it, -0.5; if a solid node or the
   end of the line comes first there is none (NaN).
2. Bridge radius: for a line that starts at the first fluid node above the
   surface and runs along the surface normal, b = crossing + 0.5 (the wall
   sits half a node before the start node).
3. Exponent: least-squares slope of log b against log t over the samples
   inside the fitting window.
"""
from __future__ import annotations

import math

import numpy as np


def line_crossing(rhoA, mask, x0, y0, dx, dy, length, level=0.5):
    """Step 1: interpolated crossing position in node steps, -0.5, or NaN."""
    a = np.asarray(rhoA, dtype=np.float64)
    m = np.asarray(mask)
    ny, nx = a.shape
    prev = None
    for k in range(length):
        x, y = x0 + k * dx, y0 + k * dy
        if not (0 <= x < nx and 0 <= y < ny) or m[y, x]:
            return math.nan
        r = a[y, x]
        if r < level:
            if prev is None:
                return -0.5
            return (k - 1) + (prev - level) / (prev - r)
        prev = r
    return math.nan


def bridge_radius(rhoA, mask, x0, y0, dx=0, dy=1, length=None, level=0.5):
    """Step 2: distance from the half-way wall to the interface along the line."""
    if length is None:
        length = np.asarray(rhoA).shape[0] - y0
    return line_crossing(rhoA, mask, x0, y0, dx, dy, length, level) + 0.5


def fit_exponent(t, b, lo, hi):
    """Step 3: slope of log b versus log t over samples with lo <= b <= hi, t > 0."""
    t = np.asarray(t, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sel = (t > 0) & np.isfinite(b) & (b >= lo) & (b <= hi)
    if sel.sum() < 3:
        return math.nan
    slope, _ = np.polyfit(np.log(t[sel]), np.log(b[sel]), 1)
    return float(slope)
