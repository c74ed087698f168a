"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the method's arithmetic: it only produces
experiment parameters (grid sizes, wall angles, radii, wetting parameters)
and initial density fields, following the set-ups of the paper's Sections 3
and 4.  The wall mask rasters, the classification and every step of the
update are computed by the oracle on one side and by the HIP library on the
other, each from its own code.

Angles are passed to both sides in radians, already converted here, so that
the two rasters receive the same double.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

MC, LLKC, IMPROVED, FIXED = 0, 1, 2, 3
BC_NAMES = {MC: "martys-chen", LLKC: "llkc", IMPROVED: "improved", FIXED: "fixed-virtual"}


@dataclass
class Case:
    """One simulation: geometry recipe, parameters and initial densities."""

    name: str
    nx: int
    ny: int
    periodic: int = 0           # bit0 x, bit1 y
    tau: float = 1.0
    G: float = 0.9
    bc: int = MC
    Gw: float = 0.0
    chiA: float = 1.0
    chiB: float = 1.0
    avg: int = 0                # 0 = D2Q25 average, 1 = D2Q9 average
    steps: int = 100
    # geometry recipe: ("rows", (y...)) | ("plane", beta_rad, R0) | ("disk", cx, cy, R) | ("none",)
    geometry: tuple = ("none",)
    rhoA0: np.ndarray | None = field(default=None, repr=False)
    rhoB0: np.ndarray | None = field(default=None, repr=False)
    mask_user: np.ndarray | None = field(default=None, repr=False)
    model: int = 0              # 0 = two components, 1 = single-component multiphase
    rho0: float = 1.0           # single-component pseudopotential density scale

    def params(self) -> dict:
        d = dict(tau=self.tau, G=self.G, bc=self.bc, Gw=self.Gw, chiA=self.chiA,
                 chiB=self.chiB, avg=self.avg, periodic=self.periodic)
        if self.model:
            d.update(model=self.model, rho0=self.rho0)
        return d


def rows_mask(nx: int, ny: int, rows) -> np.ndarray:
    """A user mask with whole solid rows (on-grid walls)."""
    m = np.zeros((ny, nx), np.uint8)
    for r in rows:
        m[r, :] = 1
    return m


def sharp_drop(nx, ny, cx, cy, R, rho_in=1.0, rho_out=0.03):
    """Sharp circular drop of A in B (Section 3.1): inclusive circle."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    inside = (xx - cx) ** 2 + (yy - cy) ** 2 <= R * R
    rA = np.where(inside, rho_in, rho_out).astype(np.float64)
    rB = np.where(inside, rho_out, rho_in).astype(np.float64)
    return rA, rB


def tanh_two_drops(nx, ny, xc1, xc2, yc, R0, rho1=1.0, rho2=0.055, delta=8.0):
    """Two drops with smoothed interfaces, the initial condition of Section 4."""
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    h1 = 0.5 * (rho1 - rho2) * (1.0 - np.tanh(((xx - xc1) ** 2 + (yy - yc) ** 2 - R0 * R0) / delta ** 2))
    h2 = 0.5 * (rho1 - rho2) * (1.0 - np.tanh(((xx - xc2) ** 2 + (yy - yc) ** 2 - R0 * R0) / delta ** 2))
    rA = rho2 + h1 + h2
    rB = rho1 - h1 - h2
    return rA, rB


def random_mixture(nx, ny, seed, mean=0.5, amp=0.01):
    """Near-uniform 50/50 mixture with seeded noise (spinodal start)."""
    rng = np.random.default_rng(seed)
    d = amp * (2.0 * rng.random((ny, nx)) - 1.0)
    return mean + d, mean - d


# ---------------------------------------------------------------------------
# The five configurations and the out-of-cache roofline grid
# ---------------------------------------------------------------------------

def config1(G=0.9) -> Case:
    """64x64, periodic in x, on-grid walls y=0,63, half drop R=15 on the bottom wall, Martys-Chen."""
    nx = ny = 64
    rA, rB = sharp_drop(nx, ny, 32.0, 0.5, 15.0, 1.0, 0.03)
    return Case("c1-flat-wall-64x64-mc", nx, ny, periodic=1, tau=1.0, G=G, bc=MC, Gw=-0.2,
                steps=2000, geometry=("rows", (0, ny - 1)), rhoA0=rA, rhoB0=rB,
                mask_user=rows_mask(nx, ny, (0, ny - 1)))


def plane_drop(nx, ny, beta_deg, R0, bc, *, G=0.9, tau=1.0, rho_out=0.03, Gw=None, chi=(1.0, 1.0),
               steps=100, name=None) -> Case:
    """Drop of radius R0 at the box centre, tangent to a plane inclined by beta (Section 3.1)."""
    beta = math.radians(beta_deg)
    rA, rB = sharp_drop(nx, ny, nx / 2.0, ny / 2.0, R0, 1.0, rho_out)
    if Gw is None:
        Gw = {MC: -0.2, LLKC: -0.5, IMPROVED: 0.0, FIXED: 0.0}[bc]
    return Case(name or "plane-%dx%d-b%g-%s" % (nx, ny, beta_deg, BC_NAMES[bc]), nx, ny, periodic=0,
                tau=tau, G=G, bc=bc, Gw=Gw, chiA=chi[0], chiB=chi[1], steps=steps,
                geometry=("plane", beta, float(R0)), rhoA0=rA, rhoB0=rB)


# Single-component multiphase Shan-Chen (psi = 1 - exp(-rho)) at G = -5: the
# flat-interface coexistence densities of that model (vapour, liquid).
SC1_G = -5.0
SC1_RHO_V, SC1_RHO_L = 0.1194, 1.8884


def sc1_plane_drop(nx, ny, beta_deg, R0, bc, *, Gw=None, G=SC1_G, tau=1.0, steps=100, name=None) -> Case:
    """Liquid drop in its vapour, tangent to a plane inclined by beta (Section 3.1
    set-up) in the single-component model; Martys-Chen G_w = -3 and LLKC
    G_w = -5 give contact angles near 70 degrees on a flat wall."""
    beta = math.radians(beta_deg)
    rA, _ = sharp_drop(nx, ny, nx / 2.0, ny / 2.0, R0, SC1_RHO_L, SC1_RHO_V)
    if Gw is None:
        Gw = {MC: -3.0, LLKC: -5.0}[bc]
    return Case(name or "sc1-plane-%dx%d-b%g-%s" % (nx, ny, beta_deg, BC_NAMES[bc]), nx, ny, periodic=0,
                tau=tau, G=G, bc=bc, Gw=Gw, steps=steps, geometry=("plane", beta, float(R0)), rhoA0=rA,
                rhoB0=None, model=1)


def config2() -> Case:
    """512x256, 30 degree stair wall, drop R=40, improved scheme (chi = 1), FP32, 20k steps."""
    return plane_drop(512, 256, 30.0, 40.0, IMPROVED, steps=20000,
                      name="c2-plane30-512x256-improved")


def config3(seed: int = 0) -> Case:
    """1024x1024, solid disk R=300 at the centre, two tanh drops R0=60 touching on top."""
    nx = ny = 1024
    rng = np.random.default_rng(seed)
    s = float(rng.uniform(0.3, 0.7))          # solid density of the run
    cx, cy, Rs, R0 = 512.0, 512.0, 300.0, 60.0
    theta = math.radians(71.0)
    top = cy + Rs
    xc1 = cx - R0 * math.sin(theta) - 1.0
    xc2 = cx + R0 * math.sin(theta) + 1.0
    yc = top - R0 * math.cos(theta)
    rA, rB = tanh_two_drops(nx, ny, xc1, xc2, yc, R0, 1.0, 0.03, 8.0)
    return Case("c3-disk-1024-improved-seed%d" % seed, nx, ny, periodic=0, tau=1.0, G=0.9,
                bc=IMPROVED, chiA=2.0 * s, chiB=2.0 - 2.0 * s, steps=50000,
                geometry=("disk", cx, cy, Rs), rhoA0=rA, rhoB0=rB)


def coalescence(R0: float, Rs: float | None = None, *, Oh=0.286, sigma=0.026, theta_deg=71.0, xi=-0.2,
                rho1=1.0, rho2=0.055, delta=8.0, G=3.0, steps=None, aspect=(14.0, 10.0)) -> Case:
    """Two drops coalescing on a flat (Rs None) or circular surface (Section 4).

    Box L_X x L_Y = 14 R0 x 10 R0; the surface passes through (L_X/2, L_Y/2)
    (flat: solid on or below y = L_Y/2; curved: the disk of radius Rs centred
    at (L_X/2, L_Y/2 - Rs)); tanh drops of radius R0 placed at contact angle
    theta against it, 2 nodes apart at the surface.  The viscosity follows
    from the Ohnesorge number, nu = Oh sqrt(sigma R0) with rho = 1 and the
    surface tension sigma of the Laplace test at G = 3; tau = 3 nu + 1/2.
    Improved scheme with the wetting parameter xi read as chi^A = 1 - xi,
    chi^B = 1 + xi (the reading under which xi = -0.2 gives the paper's
    71 degrees and xi < 0 wets the drop fluid).  steps defaults to four
    viscous times tau_nu = nu R0 / sigma."""
    nx, ny = int(round(aspect[0] * R0)), int(round(aspect[1] * R0))
    th = math.radians(theta_deg)
    xc1 = nx / 2.0 - R0 * math.sin(th) - 1.0
    xc2 = nx / 2.0 + R0 * math.sin(th) + 1.0
    yc = ny / 2.0 - R0 * math.cos(th)
    rA, rB = tanh_two_drops(nx, ny, xc1, xc2, yc, R0, rho1, rho2, delta)
    nu = Oh * math.sqrt(sigma * R0)
    tau = 3.0 * nu + 0.5
    t_nu = nu * R0 / sigma
    if Rs is None:
        geom = ("plane", 0.0, 0.0)
    else:
        geom = ("disk", nx / 2.0, ny / 2.0 - Rs, float(Rs))
    name = "coalescence-R0%g-%s-%dx%d" % (R0, "flat" if Rs is None else "Rs%g" % Rs, nx, ny)
    c = Case(name, nx, ny, periodic=0, tau=tau, G=G, bc=IMPROVED, chiA=1.0 - xi, chiB=1.0 + xi,
             steps=int(steps if steps is not None else round(4 * t_nu)), geometry=geom, rhoA0=rA, rhoB0=rB)
    c.t_nu = t_nu
    c.R0 = float(R0)
    return c


def config4_instances(n: int = 64, seed0: int = 0):
    """Batch of seeded instances: W in 128..768, H in 64..384, beta in [0, 45] degrees."""
    out = []
    for s in range(seed0, seed0 + n):
        rng = np.random.default_rng(1000 + s)
        W = int(rng.integers(128, 769))
        H = int(rng.integers(64, 385))
        beta = float(rng.uniform(0.0, 45.0))
        bc = int(rng.integers(0, 3))
        R0 = H / 5.0
        c = plane_drop(W, H, beta, R0, bc, steps=10000, name="c4-%02d-%dx%d-b%.1f-%s" % (
            s, W, H, beta, BC_NAMES[bc]))
        out.append(c)
    return out


def config5_requests(n: int = 400, seed: int = 12345, rate: float = 200.0):
    """Served stream: Poisson arrivals, sizes 64x64..2048x1024, 2k-20k steps, mixed BCs."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        W = int(rng.integers(64, 2049))
        H = int(rng.integers(64, 1025))
        steps = int(rng.integers(2000, 20001))
        beta = float(rng.uniform(0.0, 45.0))
        bc = int(rng.integers(0, 3))
        R0 = max(4.0, H / 5.0)
        c = plane_drop(W, H, beta, R0, bc, steps=steps, name="c5-%03d" % k)
        reqs.append((t, c))
    return reqs


def sc1_roofline_case(nx=5600, ny=4000, seed=7) -> Case:
    """The same grid for the single-component model: a seeded near-uniform
    density inside the spinodal region at G = -5 (it separates into liquid
    and vapour), fully periodic."""
    rng = np.random.default_rng(seed)
    rA = 0.7 + 0.02 * (2.0 * rng.random((ny, nx)) - 1.0)
    return Case("r-sc1-periodic-%dx%d" % (nx, ny), nx, ny, periodic=3, tau=1.0, G=SC1_G, bc=MC, Gw=0.0,
                steps=1000, geometry=("none",), rhoA0=rA, rhoB0=None, model=1,
                mask_user=np.zeros((ny, nx), np.uint8))


def roofline_case(nx=5600, ny=4000, seed=7, G=3.0) -> Case:
    """The paper's largest grid (Section 4 convergence study) as a fully periodic mixture."""
    rA, rB = random_mixture(nx, ny, seed)
    return Case("r-periodic-%dx%d" % (nx, ny), nx, ny, periodic=3, tau=1.0, G=G, bc=MC, Gw=0.0,
                steps=1000, geometry=("none",), rhoA0=rA, rhoB0=rB,
                mask_user=np.zeros((ny, nx), np.uint8))


def roofline_plane_case(bc, nx=5600, ny=4000, beta_deg=30.0, R0=400.0) -> Case:
    """The paper's largest grid (Section 4) with the Section 3.1 set-up: a drop
    of radius 400 at rest on a 30-degree stair plane, G = 3, rho 1.0/0.055, in
    each wetting rule (Martys-Chen G_w = -0.2, LLKC G_w = -0.5, improved scheme
    chi^A = 1.2, chi^B = 0.8): the out-of-cache rows of the wall rules."""
    return plane_drop(nx, ny, beta_deg, R0, bc, G=3.0, rho_out=0.055, chi=(1.2, 0.8),
                      name="r-plane%g-%dx%d-%s" % (beta_deg, nx, ny, BC_NAMES[bc]))


def input_hash(c: Case, mask) -> str:
    """Fingerprint of a case's inputs (wall mask, initial densities,
    parameters), so that stored expected values can be matched to them."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(mask, np.uint8).tobytes())
    h.update(np.ascontiguousarray(c.rhoA0, np.float64).tobytes())
    h.update(np.ascontiguousarray(c.rhoB0, np.float64).tobytes())
    h.update(repr(sorted(c.params().items())).encode())
    return h.hexdigest()[:16]
