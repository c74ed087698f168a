"""Device contact-angle measurement (lbm_contour_fit) against the oracle's.

The device reduces the interface points of the FP32 density field in FP64 on
the GPU; the oracle measures its own FP64 field with its own code.  Same
seeded inputs on both sides.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _sim(case, mask, **kw):
    from paper_2009_12584_amd.sim import Simulation

    return Simulation(mask, case.rhoA0, case.rhoB0, **case.params(), **kw)


def _cap_case(nx=200, ny=160, y0=30, R=40.0, theta=71.0):
    yw = y0 + 0.5
    xc, yc = nx / 2 + 0.3, yw - R * math.cos(math.radians(theta))
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    rA = 0.055 + (1.0 - 0.055) * (0.5 + 0.5 * np.tanh((R - np.hypot(xx - xc, yy - yc)) / 2.0))
    m = np.zeros((ny, nx), np.uint8)
    m[: y0 + 1, :] = 1
    m[:, 0] = m[:, -1] = 1
    m[-1, :] = 1
    c = W.Case("cap", nx, ny, tau=1.0, G=3.0, bc=W.MC, Gw=-0.2, rhoA0=rA, rhoB0=1.055 - rA)
    return c, m, (xc, yc, R)


def test_contour_fit_of_a_known_cap_at_step_zero(ora):
    from oracle import contact_angle as CA

    level = 0.5275  # half-way between the two bulk densities of the cap
    c, m, (xc, yc, R) = _cap_case()
    s = _sim(c, m)
    print("case: cap 200x160 step 0", flush=True)
    g = s.contour_fit(level, 3)
    ref = CA.measure(c.rhoA0, m, level=level, skip=3)
    s.close()
    assert g["n"] == ref["n"]
    for k in ("xc", "yc", "R"):
        assert g[k] == pytest.approx(ref[k], abs=1e-4), k
    assert g["rms"] == pytest.approx(ref["rms"], abs=1e-4)
    assert (g["xc"], g["yc"], g["R"]) == (pytest.approx(xc, abs=0.03), pytest.approx(yc, abs=0.03),
                                        pytest.approx(R, abs=0.03))


@pytest.mark.parametrize("bc,kw", [(W.MC, dict(Gw=-0.2)), (W.IMPROVED, dict(chi=(1.2, 0.8)))],
                         ids=["martys-chen", "improved-xi-0.2"])
def test_contact_angle_matches_the_oracle_after_4500_steps(ora, bc, kw):
    from oracle import contact_angle as CA
    from paper_2009_12584_amd import analysis as A

    nx, ny, R0, steps = 128, 112, 16.0, 4500
    c = W.plane_drop(nx, ny, 0.0, R0, bc, G=3.0, rho_out=0.055, **kw)
    from paper_2009_12584_amd.sim import mask_plane

    m = mask_plane(nx, ny, c.geometry[1], c.geometry[2])
    print("case: plane drop %s %dx%d %d steps" % (W.BC_NAMES[bc], nx, ny, steps), flush=True)
    s = _sim(c, m)
    s.step(steps)
    g = s.contour_fit(0.5, 3)
    s.close()
    o = ora.Oracle(ora.mask_plane(nx, ny, c.geometry[1], c.geometry[2]), c.rhoA0, c.rhoB0, **c.params())
    o.step(steps)
    ref = CA.measure(o.fields()[0], ora.mask_plane(nx, ny, c.geometry[1], c.geometry[2]), skip=3)
    th = A.contact_angle(g, A.wall_line(m))
    assert abs(g["n"] - ref["n"]) <= 2
    assert g["R"] == pytest.approx(ref["R"], abs=5e-3)
    assert th == pytest.approx(ref["theta"], abs=0.05)


def test_batch_contour_fit_equals_single(ora):
    from paper_2009_12584_amd.sim import Batch, mask_plane

    cases = [W.plane_drop(140, 120, b, 16.0, W.IMPROVED, G=3.0, rho_out=0.055, chi=(1.1, 0.9)) for b in (0.0, 30.0)]
    masks = [mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]
    print("case: batch of 2 plane drops, 600 steps", flush=True)
    b = Batch([(m, c.rhoA0, c.rhoB0, c.params()) for c, m in zip(cases, masks)])
    b.step(600)
    got = [b.contour_fit(i, 0.5, 3, (10, 10, 129, 109)) for i in range(2)]
    b.close()
    for i, (c, m) in enumerate(zip(cases, masks)):
        s = _sim(c, m)
        s.step(600)
        ref = s.contour_fit(0.5, 3, (10, 10, 129, 109))
        s.close()
        assert got[i] == ref


def test_contour_fit_rejects_bad_requests(ora):
    from paper_2009_12584_amd.capi import LBM_EINVAL, LbmError

    c, m, _ = _cap_case(80, 70, 10, 15.0, 90.0)
    s = _sim(c, m)
    print("case: contour fit argument checks", flush=True)
    for kw in (dict(level=float("nan")), dict(skip=33), dict(skip=-1), dict(roi=(0, 0, 80, 10)),
               dict(roi=(5, 5, 4, 10)), dict(roi=(-1, 0, 10, 10))):
        with pytest.raises(LbmError) as e:
            s.contour_fit(**kw)
        assert e.value.code == LBM_EINVAL
    # a region without interface gives no circle, not an error
    r = s.contour_fit(0.5, 0, (1, 60, 20, 68))
    assert r["n"] == 0 and math.isnan(r["R"])
    s.close()


def test_theta_of_xi_on_flat_and_inclined_walls(ora):
    """Improved scheme, small drops: neutral at xi = 0, the paper's sign for
    xi != 0 with chi = (1 - xi, 1 + xi), and a small spread over the wall
    inclination (Section 3.2)."""
    from paper_2009_12584_amd import analysis as A

    print("case: theta(xi, beta) sweep 220x220 R0=22 8000 steps", flush=True)
    rows = A.sweep([-0.2, 0.0, 0.2], [0.0, 30.0], [0], n=220, R0=22.0, tau=1.0, steps=8000, checkpoints=2,
                   chunk=4000)
    th = {(r["beta"], r["xi"]): r["theta"][-1] for r in rows}
    for beta in (0.0, 30.0):
        assert th[(beta, 0.0)] == pytest.approx(90.0, abs=2.5)
        assert th[(beta, -0.2)] < 80.0
        assert th[(beta, 0.2)] > 100.0
    # small drops, not yet at rest: the inclined stair shifts the angle by a few degrees
    for xi in (-0.2, 0.0, 0.2):
        assert abs(th[(0.0, xi)] - th[(30.0, xi)]) < 6.0
