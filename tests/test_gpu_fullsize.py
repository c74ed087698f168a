"""Parity at the full sizes the benchmark times, on sampled windows.

After k steps the state of a node depends only on the initial state within
4 k nodes: one node of streaming per step plus at most three of the force
stencil (the improved scheme averages over the two belts around a solid
node one node away; the other forces reach one node).  So the oracle can
check a full-size GPU run on windows: it runs each window of the initial
state, wrapped periodically, for k steps, and the window's interior more
than 4 k nodes from its edge must match the GPU's full-grid result to the
same bar as the small parity cases.  The GPU runs in the launch shape the
benchmark times for that grid.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5
U_TOL = 1e-6
K = 10
MARGIN = 4 * K + 2
SIZE = 240


def _errors(fl, g, r, two):
    er = np.max(np.abs(g[0] - r[0])[fl] / r[0][fl])
    if two:
        er = max(er, np.max(np.abs(g[1] - r[1])[fl] / r[1][fl]))
    eu = max(np.max(np.abs(g[2] - r[2])[fl]), np.max(np.abs(g[3] - r[3])[fl]))
    return er, eu


def _window_check(ora, c, mask, fields, windows, tol):
    two = c.model == 0
    for (x0, y0) in windows:
        xs = (np.arange(SIZE) + x0) % c.nx
        ys = (np.arange(SIZE) + y0) % c.ny
        cut = np.ix_(ys, xs)
        prm = c.params()
        prm["periodic"] = 3
        o = ora.Oracle(mask[cut], c.rhoA0[cut], c.rhoB0[cut] if two else None, **prm)
        o.step(K)
        of = o.fields()
        sl = (slice(MARGIN, SIZE - MARGIN),) * 2
        fl = mask[cut][sl] == 0
        er, eu = _errors(fl, [f[cut][sl] for f in fields], [f[sl] for f in of], two)
        print("  window at (%d,%d): rel rho %.2e abs u %.2e over %d fluid nodes" % (x0, y0, er, eu, fl.sum()),
              flush=True)
        assert fl.sum() > 0
        assert er <= tol[0] and eu <= tol[1], (x0, y0, er, eu)


def _run(c, mask, storage, ty, lanes):
    from paper_2009_12584_amd.sim import Simulation

    print("case: %s %s, %d steps, tile rows %d, lanes %d" % (c.name, storage, K, ty, lanes), flush=True)
    s = Simulation(mask, c.rhoA0, c.rhoB0 if c.model == 0 else None, storage=storage, tile_y=ty, lanes=lanes,
                   **c.params())
    s.step(K)
    f = s.fields()
    s.close()
    return f


# windows across both periodic seams, one in the bulk, one on the x seam
SEAMS = [(5600 - 120, 4000 - 120), (2800, 1900), (5500, 700)]


@pytest.mark.parametrize("storage,tol", [("f32", (RHO_TOL, U_TOL)), ("f16", (5e-3, 1e-3))], ids=["f32", "f16"])
def test_roofline_mixture_5600x4000_windows(ora, storage, tol):
    """The 5600 x 4000 periodic G = 3 mixture (Martys-Chen path), one lane,
    64 x 8 tiles: the out-of-cache roofline row."""
    c = W.roofline_case()
    f = _run(c, c.mask_user, storage, 8, 1)
    _window_check(ora, c, c.mask_user, f, SEAMS, tol)


def test_single_component_5600x4000_windows(ora):
    """The 5600 x 4000 periodic single-component case at G = -5, 64 x 8 tiles."""
    c = W.sc1_roofline_case()
    f = _run(c, c.mask_user, "f32", 8, 1)
    _window_check(ora, c, c.mask_user, f, SEAMS, (RHO_TOL, U_TOL))


@pytest.mark.parametrize("lanes", [1, 2])
def test_improved_plane_5600x4000_windows(ora, lanes):
    """The same grid with a 30-degree stair wall, a drop of radius 400 and the
    improved scheme: windows on the contact line, on the bare wall and in the
    bulk, in both lane layouts."""
    from paper_2009_12584_amd.sim import mask_plane

    c = W.plane_drop(5600, 4000, 30.0, 400.0, W.IMPROVED, G=3.0, rho_out=0.055, chi=(1.2, 0.8))
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    f = _run(c, m, "f32", 8, lanes)
    # the drop touches the plane where the normal through the centre meets it,
    # 400 nodes below and to the side of (2800, 2000) along the 30-degree normal
    wins = [(2800 + 200 - SIZE // 2, 2000 - 346 - SIZE // 2), (600, 150), (3000, 3000)]
    for (x0, y0) in wins[:2]:
        sub = m[y0:y0 + SIZE, x0:x0 + SIZE]
        assert 0 < sub.sum() < sub.size, "window must straddle the wall"
    _window_check(ora, c, m, f, wins, (RHO_TOL, U_TOL))


@pytest.mark.parametrize("ty,lanes", [(4, 1), (8, 2)])
def test_batch_of_64_sampled_instances(ora, ty, lanes):
    """The 64-instance batch the benchmark times, one launch per step inside
    a graph; three instances re-run whole on the oracle."""
    from paper_2009_12584_amd.sim import Batch, mask_plane

    cases = W.config4_instances(64)
    masks = [mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]
    print("case: batch of 64 instances, 100 steps in graphs of 50, tile rows %d, lanes %d" % (ty, lanes),
          flush=True)
    b = Batch([(m, c.rhoA0, c.rhoB0, c.params()) for m, c in zip(masks, cases)], tile_y=ty, lanes=lanes,
              graph_steps=50)
    b.step(100)
    try:
        for k in (0, 29, 63):
            g = b.fields(k)
            o = ora.Oracle(masks[k], cases[k].rhoA0, cases[k].rhoB0, **cases[k].params())
            o.step(100)
            er, eu = _errors(masks[k] == 0, g, o.fields(), True)
            print("  instance %d %s: rel rho %.2e abs u %.2e" % (k, cases[k].name, er, eu), flush=True)
            assert er <= RHO_TOL and eu <= U_TOL, (k, er, eu)
    finally:
        b.close()
