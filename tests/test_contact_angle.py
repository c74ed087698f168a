"""Contact-angle measurement (Section 3.2) on the oracle, pinned.

1. The measurement itself against closed-form drops: a smooth circular cap of
   known centre and radius on a flat and on an inclined stair wall must come
   back with its own circle and angle.
2. The oracle's static drops against symmetry and against the paper:
   - neutral walls (G_w = 0, or chi = 1) give 90 degrees (the A/B swap maps
     the drop onto its complement, Section 2 after Eq. 7);
   - swapping the sign of the wetting parameter mirrors the angle about the
     neutral one (same swap);
   - the angles the paper prints for its parameters (55 and 63 degrees for
     Martys-Chen and LLKC, approximate in the paper; 71 degrees for the
     improved scheme at xi = -0.2), with the tolerance stated per case;
   - the sign of xi: with chi^A = 1 - xi, chi^B = 1 + xi in Eq. 7's literal
     reading, xi < 0 is hydrophilic as the paper states; the literal
     chi^A = 1 + xi gives the mirror angle.
The host helpers of the product's analysis module (wall line, angle) are
checked against the same closed forms; they share no code with the oracle's.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _cap_field(nx, ny, xc, yc, R, width=2.0):
    """rho^A = 0.5 exactly on the circle, smooth tanh profile across it."""
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(xx - xc, yy - yc)
    return 0.5 + 0.5 * np.tanh((R - r) / width)


def _flat_mask(nx, ny, y0):
    m = np.zeros((ny, nx), np.uint8)
    m[: y0 + 1, :] = 1
    m[:, 0] = m[:, -1] = 1
    m[-1, :] = 1
    return m


@pytest.mark.parametrize("theta", [45.0, 71.0, 90.0, 120.0])
def test_measure_recovers_a_known_cap_on_a_flat_wall(ora, theta):
    from oracle import contact_angle as CA

    nx, ny, y0, R = 200, 160, 30, 40.0
    yw = y0 + 0.5  # bounce-back wall half-way above the top solid row
    xc, yc = 100.0, yw - R * math.cos(math.radians(theta))
    m = _flat_mask(nx, ny, y0)
    r = CA.measure(_cap_field(nx, ny, xc, yc, R), m, skip=3)
    assert r["theta"] == pytest.approx(theta, abs=0.05)
    # linear interpolation along edges oblique to the interface: ~1e-2 nodes
    assert r["R"] == pytest.approx(R, abs=0.02)
    assert (r["xc"], r["yc"]) == (pytest.approx(xc, abs=0.02), pytest.approx(yc, abs=0.02))
    assert r["rms"] < 0.01


@pytest.mark.parametrize("beta", [20.0, 45.0])
def test_measure_recovers_a_known_cap_on_an_inclined_stair_wall(ora, beta):
    from oracle import contact_angle as CA

    n, R0, theta, R = 240, 30.0, 71.0, 45.0
    b = math.radians(beta)
    m = ora.mask_plane(n, n, b, R0)
    # the plane of Section 3.1 (solid on or below it)
    x0, y0 = n / 2 + R0 * math.sin(b), n / 2 - R0 * math.cos(b)
    # circle centre at height -R cos(theta) above the line, over the tangent point
    nrm = np.array([-math.sin(b), math.cos(b)])
    c = np.array([x0, y0]) + nrm * (-R * math.cos(math.radians(theta)))
    r = CA.measure(_cap_field(n, n, c[0], c[1], R), m, skip=3, roi=(20, 20, n - 21, n - 21))
    # the stair's half-way points scatter about the line by less than half a node
    assert r["theta"] == pytest.approx(theta, abs=0.8)
    assert r["R"] == pytest.approx(R, abs=0.02)
    a, bb = CA.wall_line(m)
    assert a == pytest.approx(math.tan(b), rel=2e-3)


def test_product_host_helpers_agree_with_the_closed_form(ora):
    from oracle import contact_angle as CA
    from paper_2009_12584_amd import analysis as A

    m = _flat_mask(120, 90, 20)
    assert A.wall_line(m) == pytest.approx((0.0, 20.5), abs=1e-12)
    for beta in (10.0, 30.0, 60.0):
        mp = ora.mask_plane(300, 300, math.radians(beta), 40.0)
        assert A.wall_line(mp) == pytest.approx(CA.wall_line(mp), abs=1e-9)
    wall = (0.0, 20.5)
    assert A.contact_angle(dict(xc=50.0, yc=20.5, R=10.0), wall) == pytest.approx(90.0, abs=1e-12)
    assert A.contact_angle(dict(xc=50.0, yc=20.5 - 5.0, R=10.0), wall) == pytest.approx(60.0, abs=1e-9)
    assert A.contact_angle(dict(xc=50.0, yc=20.5 + 5.0, R=10.0), wall) == pytest.approx(120.0, abs=1e-9)
    assert A.xi_to_chi(-0.2) == pytest.approx((1.2, 0.8))


# ---------------------------------------------------------------- static drops on the oracle

NX, NY, R0, STEPS = 128, 112, 16.0, 4500

CASES = {
    "mc0": (W.MC, dict(Gw=0.0)),
    "mc-": (W.MC, dict(Gw=-0.2)),
    "mc+": (W.MC, dict(Gw=+0.2)),
    "llkc-": (W.LLKC, dict(Gw=-0.5)),
    "imp1": (W.IMPROVED, dict(chi=(1.0, 1.0))),
    "imp-xi": (W.IMPROVED, dict(chi=(1.2, 0.8))),   # xi = -0.2 with chi^A = 1 - xi
    "imp-lit": (W.IMPROVED, dict(chi=(0.8, 1.2))),  # xi = -0.2 with chi^A = 1 + xi
    "fix=": (W.FIXED, dict(chi=(0.5, 0.5))),        # rho_s^A = rho_s^B
    "fixA": (W.FIXED, dict(chi=(0.7, 0.3))),        # solid looks A-rich
    "fixB": (W.FIXED, dict(chi=(0.3, 0.7))),
}


@pytest.fixture(scope="module")
def angles(ora):
    from oracle import contact_angle as CA

    out = {}
    for key, (bc, kw) in CASES.items():
        c = W.plane_drop(NX, NY, 0.0, R0, bc, G=3.0, rho_out=0.055, **kw)
        m = ora.mask_plane(NX, NY, c.geometry[1], c.geometry[2])
        o = ora.Oracle(m, c.rhoA0, c.rhoB0, **c.params())
        o.step(STEPS)
        out[key] = CA.measure(o.fields()[0], m, skip=3)
        del o
    return out


def test_static_drops_are_circular(angles):
    for key, r in angles.items():
        assert r["n"] > 60, key
        assert r["rms"] < 0.02, key


def test_neutral_walls_give_ninety_degrees(angles):
    target = GOLDEN["neutral_wetting_chi_1_deg"]["value"]
    # the extrapolated circle sits about half a node off the half-way wall at R ~ 22
    assert angles["mc0"]["theta"] == pytest.approx(target, abs=2.0)
    assert angles["imp1"]["theta"] == pytest.approx(target, abs=2.0)


def test_opposite_wetting_mirrors_the_angle(angles):
    a = angles
    assert a["mc-"]["theta"] + a["mc+"]["theta"] == pytest.approx(2 * a["mc0"]["theta"], abs=1.0)
    assert a["imp-xi"]["theta"] + a["imp-lit"]["theta"] == pytest.approx(2 * a["imp1"]["theta"], abs=1.0)
    assert a["mc-"]["theta"] < 80.0 < 100.0 < a["mc+"]["theta"]


def test_martys_chen_and_llkc_angles_near_the_printed_ones(angles):
    # the paper gives these as approximate values and states neither tau nor the
    # measurement for them; halving, doubling or flipping G_w moves the angle by
    # more than 10 degrees out of the band (oracle: 78, 33, 118 degrees for MC)
    mc = GOLDEN["contact_angle_mc_gw_m0.2_deg"]["value"]
    llkc = GOLDEN["contact_angle_llkc_gw_m0.5_deg"]["value"]
    assert angles["mc-"]["theta"] == pytest.approx(mc, abs=10.0)
    assert angles["llkc-"]["theta"] == pytest.approx(llkc, abs=10.0)
    assert angles["mc-"]["theta"] < angles["llkc-"]["theta"] < 90.0


def test_fixed_virtual_density_wets_the_component_it_mimics(angles):
    """Chen et al.'s constant solid densities (Section 2): equal densities are
    neutral by the A/B swap; an A-rich solid attracts A, and swapping the two
    densities mirrors the angle."""
    a = angles
    # the depletion layer both components form at a repelling wall moves the
    # extrapolated circle by ~2 degrees at R ~ 22 (equal rho_s of 0.2 and 1.0
    # give 91.7 and 92.3 degrees); the bias falls as 1/R
    assert a["fix="]["theta"] == pytest.approx(90.0, abs=2.5)
    assert a["fixA"]["theta"] < 80.0 < 100.0 < a["fixB"]["theta"]
    assert a["fixA"]["theta"] + a["fixB"]["theta"] == pytest.approx(2 * a["fix="]["theta"], abs=1.0)


def test_xi_sign_matches_the_paper_with_chi_a_one_minus_xi(angles):
    target = GOLDEN["contact_angle_improved_xi_m0.2_deg"]["value"]
    # R0 = 16 here against R0 = 100 in the paper
    assert angles["imp-xi"]["theta"] == pytest.approx(target, abs=6.0)
    assert angles["imp-lit"]["theta"] > 100.0
