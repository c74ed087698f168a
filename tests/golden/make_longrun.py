"""Writes the FP64 oracle's fields after the configurations' full runs, on
sampled nodes, for the GPU parity tests at each configuration's final step.

Calls only ``oracle`` (the checker) and ``workloads`` (the seeded inputs): no
value here comes from the HIP library.  For every case it stores, at each
checkpoint, rho^A, rho^B, u_x and u_y (as float32: the rounding, 6e-8
relative, is far below the 1e-5 bar) at

  - 2048 fluid nodes drawn uniformly with a fixed seed, and
  - every fluid node of a few 24 x 24 windows placed where the method does
    its work: the contact line of a drop on the wall, the bridge between two
    coalescing drops, and the bulk.

together with a hash of the case's inputs, so a test can tell a stale file
from a changed workload.  Run from the repository root:

    python tests/golden/make_longrun.py [case ...]

Cases: c2 (512 x 256 plane, improved scheme, 20,000 steps; checkpoint 20,000),
c3 (1024 x 1024 disk, two drops, improved scheme with chi^A != chi^B, seed 0,
50,000 steps; checkpoints 1000 and 50,000), c4-00, c4-03, c4-05, c4-29 (four
instances of the 64-instance batch covering the three wetting rules, 10,000
steps).  The c3 run takes about 20 minutes on 8 cores.
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

WIN = 24
NSAMPLE = 2048


input_hash = W.input_hash


def ora_mask(c):
    g = c.geometry
    if c.mask_user is not None:
        return c.mask_user
    if g[0] == "plane":
        return oracle.mask_plane(c.nx, c.ny, g[1], g[2])
    return oracle.mask_disk(c.nx, c.ny, g[1], g[2], g[3])


def plane_contact(c):
    """The node where a drop tangent to the plane of Section 3.1 touches it."""
    beta, R0 = c.geometry[1], c.geometry[2]
    return c.nx / 2.0 + R0 * math.sin(beta), c.ny / 2.0 - R0 * math.cos(beta)


def outer_crossing(cx, cy, Rs, xd, yd, R0):
    """Leftmost crossing of the drop circle (xd, yd, R0) with the disk (cx, cy, Rs)."""
    best = None
    for k in range(36000):
        a = 2 * math.pi * k / 36000
        x, y = xd + R0 * math.cos(a), yd + R0 * math.sin(a)
        if abs(math.hypot(x - cx, y - cy) - Rs) < 0.05 and (best is None or x < best[0]):
            best = (x, y)
    return best


def sample_indices(mask, centres, seed):
    ny, nx = mask.shape
    fluid = np.flatnonzero(mask.ravel() == 0)
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(fluid, size=min(NSAMPLE, fluid.size), replace=False).tolist())
    for (cx, cy) in centres:
        x0 = int(round(cx)) - WIN // 2
        y0 = int(round(cy)) - WIN // 2
        for y in range(max(0, y0), min(ny, y0 + WIN)):
            for x in range(max(0, x0), min(nx, x0 + WIN)):
                if mask[y, x] == 0:
                    pick.add(y * nx + x)
    return np.array(sorted(pick), np.int64)


def cases():
    out = {}
    c2 = W.config2()
    out["c2"] = (c2, [c2.steps], [plane_contact(c2), (150.0, 200.0)])
    c3 = W.config3(0)
    cx, cy, Rs = c3.geometry[1], c3.geometry[2], c3.geometry[3]
    top = cy + Rs
    # the outer contact lines of the two drops (where their initial circles
    # of radius 60 cross the disk), the bridge above the disk's top, the bulk
    xl, yl = outer_crossing(cx, cy, Rs, 512.0 - 60.0 * math.sin(math.radians(71.0)) - 1.0, top - 60.0 * math.cos(
        math.radians(71.0)), 60.0)
    out["c3"] = (c3, [1000, c3.steps], [(xl, yl), (2 * cx - xl, yl), (cx, top + 4.0), (200.0, 200.0)])
    b = W.config4_instances(64)
    for k in (0, 3, 5, 29):
        out["c4-%02d" % k] = (b[k], [b[k].steps], [plane_contact(b[k])])
    return out


def run(name, c, checkpoints, centres):
    mask = ora_mask(c)
    idx = sample_indices(mask, centres, seed=2024)
    o = oracle.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    data = {"name": np.array(c.name), "nx": np.int64(c.nx), "ny": np.int64(c.ny), "idx": idx,
            "steps": np.array(checkpoints, np.int64), "input_sha": np.array(input_hash(c, mask)),
            "oracle_threads": np.int64(oracle.threads())}
    t0 = time.time()
    for T in checkpoints:
        o.step(T - o.t)
        f = o.fields()
        for key, v in zip(("rhoA", "rhoB", "ux", "uy"), f):
            data["%s_%d" % (key, T)] = v.ravel()[idx].astype(np.float32)
        tot = o.totals()
        data["mass_%d" % T] = tot[:2]
        print("%s: t=%d (%.0f s)" % (name, T, time.time() - t0), flush=True)
    path = os.path.join(HERE, "longrun_%s.npz" % name)
    np.savez_compressed(path, **data)
    print("wrote", path, "%d nodes" % idx.size, flush=True)


def main(argv):
    oracle.build()
    todo = cases()
    names = argv or list(todo)
    for n in names:
        c, cps, centres = todo[n]
        run(n, c, cps, centres)


if __name__ == "__main__":
    main(sys.argv[1:])
