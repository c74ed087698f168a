"""Drop-shape measurements: the contact angle of a static drop with the
theta(xi, beta) sweep (Section 3.2), and the bridge radius of two coalescing
drops with its growth exponent (Section 4).

The paper fits a circle to the interface rho^A = 0.5 of the static drop and
takes the angle between the circle's tangent at the contact line and the
plane.  The circle comes from the device (lbm_contour_fit,
lbm_batch_contour_fit: interface points and FP64 moments are reduced on the
GPU).  This module adds the host geometry around it: the wall line of a plane
mask, the angle between circle and wall, and a driver that runs many drops as
one batch.

Reading of the wetting parameter: Eq. 7 puts chi^sigma on the virtual density
of component sigma, and Eq. 6 makes component sigma feel the other
component's virtual density.  Taken literally, chi^A = 1 + xi, chi^B = 1 - xi
makes xi < 0 hydrophobic for the drop fluid A, while Section 2 (after Eq. 7) calls xi < 0
hydrophilic and Section 4 quotes 71 degrees at xi = -0.2.  The measured
angles reproduce the paper's only with chi^A = 1 - xi, chi^B = 1 + xi, so
xi_to_chi returns that pair; the C ABI keeps chi^A, chi^B exactly as Eq. 7.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from .sim import Batch, mask_plane


def xi_to_chi(xi: float):
    """(chi^A, chi^B) for the paper's wetting parameter xi (xi < 0 wets the drop fluid A)."""
    return 1.0 - float(xi), 1.0 + float(xi)


def wall_line(mask, columns=None):
    """Least-squares line y = a x + b through the bounce-back wall of a bottom plane.

    In each column the wall sits half a node below the first fluid node above
    the bottom border row.  Columns without fluid, and those whose first fluid
    node is row 1 (the border itself is the wall there), do not count."""
    m = np.asarray(mask) != 0
    ny, nx = m.shape
    cols = np.arange(1, nx - 1) if columns is None else np.asarray(list(columns), dtype=np.int64)
    fluid = ~m[1:, cols]
    first = np.argmax(fluid, axis=0) + 1
    keep = fluid.any(axis=0) & (first > 1)
    if keep.sum() < 2:
        raise ValueError("no plane wall found in the given columns")
    a, b = np.polyfit(cols[keep].astype(np.float64), first[keep] - 0.5, 1)
    return float(a), float(b)


def contact_angle(circle, wall) -> float:
    """Angle in degrees, measured through the drop, between the circle and the
    wall y = a x + b (fluid above the wall): cos(theta) = -h / R with h the
    signed height of the circle centre above the wall."""
    a, b = wall
    h = (circle["yc"] - (a * circle["xc"] + b)) / math.sqrt(1.0 + a * a)
    return math.degrees(math.acos(max(-1.0, min(1.0, -h / circle["R"]))))


def drop_roi(nx, ny, R0, half=3.5):
    """Box around a drop started at the box centre, clipped to the interior."""
    h = int(round(half * R0))
    cx, cy = nx // 2, ny // 2
    return (max(1, cx - h), max(1, cy - h), min(nx - 2, cx + h), min(ny - 2, cy + h))


def sweep(xis, betas, avgs=(0,), *, n=1000, R0=100.0, tau=1.88, G=3.0, rho_out=0.055, steps=60000,
          checkpoints=3, chunk=2000, skip=3, extra_skips=(), storage="f32", log=None):
    """Drops of radius R0 on planes inclined by beta (Sections 3.1 and 4),
    improved virtual density with chi from xi_to_chi, all run as one batch.
    Returns one dict per (avg, beta, xi) with the angle, radius, point count
    and rms residual of the circle at each checkpoint (wall cut `skip`), and
    the angle for each wall cut in extra_skips under "theta_skip<k>"."""
    import workloads as W  # synthetic initial conditions (sharp drop tangent to the plane)

    keys, cases, walls = [], [], []
    for avg in avgs:
        for beta in betas:
            for xi in xis:
                chiA, chiB = xi_to_chi(xi)
                c = W.plane_drop(n, n, beta, R0, W.IMPROVED, G=G, tau=tau, rho_out=rho_out, chi=(chiA, chiB))
                prm = c.params()
                prm["avg"] = int(avg)
                mask = mask_plane(n, n, c.geometry[1], c.geometry[2])
                keys.append((int(avg), float(beta), float(xi)))
                cases.append((mask, c.rhoA0, c.rhoB0, prm))
                walls.append(wall_line(mask, range(max(1, n // 2 - int(2.5 * R0)), min(n - 1, n // 2 + int(2.5 * R0)))))
    roi = drop_roi(n, n, R0)
    b = Batch(cases, storage=storage)
    marks = sorted({int(round(steps * (k + 1) / checkpoints)) for k in range(checkpoints)})
    rows = [dict(avg=k[0], beta=k[1], xi=k[2], theta=[], R=[], n=[], rms=[], steps=[],
                 **{"theta_skip%d" % e: [] for e in extra_skips}) for k in keys]
    t0, done = time.perf_counter(), 0
    try:
        for m in marks:
            while done < m:
                k = min(chunk, m - done)
                b.step(k)
                done += k
                if log:
                    log("sweep: step %d of %d, %.1f s" % (done, steps, time.perf_counter() - t0))
            for i, r in enumerate(rows):
                c = b.contour_fit(i, 0.5, skip, roi)
                r["theta"].append(contact_angle(c, walls[i]))
                r["R"].append(c["R"])
                r["n"].append(c["n"])
                r["rms"].append(c["rms"])
                r["steps"].append(m)
                for e in extra_skips:
                    r["theta_skip%d" % e].append(contact_angle(b.contour_fit(i, 0.5, e, roi), walls[i]))
    finally:
        b.close()
    return rows


def surface_start(mask, x0, y_surface):
    """First fluid node above the surface point (x0, y_surface) in column x0."""
    m = np.asarray(mask)
    y = int(y_surface)
    while y < m.shape[0] and m[y, x0]:
        y += 1
    if y >= m.shape[0] - 1:
        raise ValueError("no fluid above the surface in column %d" % x0)
    return y


def bridge_history(case, mask, *, every, steps=None, level=0.5, storage="f32", tile_y=0):
    """Bridge radius b(t) of two drops coalescing on a surface (Section 4).

    The probe runs up the column x = L_X / 2 from the first fluid node above
    the surface point (L_X / 2, L_Y / 2); b is the distance from the half-way
    wall below that node to the rho^A = level crossing (0 before the bridge
    forms).  Samples are written on the device, one per `every` steps, and
    read back once.  Returns (t, b) arrays."""
    import torch

    from .sim import Simulation

    steps = case.steps if steps is None else steps
    x0 = case.nx // 2
    y0 = surface_start(mask, x0, case.ny // 2)
    length = case.ny - 1 - y0
    n = steps // every
    stream = torch.cuda.current_stream()
    buf = torch.empty(max(1, n), dtype=torch.float64, device="cuda")
    sim = Simulation(mask, case.rhoA0, case.rhoB0, stream=stream, storage=storage, tile_y=tile_y, **case.params())
    try:
        for k in range(n):
            sim.step(every)
            sim.line_probe(x0, y0, 0, 1, length, level, buf.data_ptr() + 8 * k)
        stream.synchronize()
    finally:
        sim.close()
    pos = buf[:n].cpu().numpy()
    t = every * np.arange(1, n + 1, dtype=np.float64)
    return t, pos + 0.5


def fit_exponent(t, b, lo, hi):
    """Least-squares slope of log b against log t over samples with lo <= b <= hi."""
    t = np.asarray(t, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    sel = (t > 0) & np.isfinite(b) & (b >= lo) & (b <= hi)
    if sel.sum() < 3:
        return math.nan
    return float(np.polyfit(np.log(t[sel]), np.log(b[sel]), 1)[0])


def coalescence_study(R0s, Rs=None, *, samples=400, t_end=4.0, b_lo=3.0, storage="f32", nus=None, log=None):
    """Bridge growth for each initial radius at the paper's Ohnesorge number
    (or, with nus, for each kinematic viscosity at the first radius): alpha
    fitted over b_lo <= b <= R0 / 3 (the viscous regime, which ends as b
    passes R0 / 3), time in units of tau_nu = nu R0 / sigma."""
    import workloads as W

    from .sim import mask_disk, mask_plane

    runs = [(R0, None) for R0 in R0s] if not nus else [(R0s[0], nu) for nu in nus]
    out = []
    for R0, nu in runs:
        kw = {} if nu is None else {"Oh": nu / math.sqrt(0.026 * R0)}
        c = W.coalescence(R0, Rs, **kw)
        steps = int(round(t_end * c.t_nu))
        every = max(1, steps // samples)
        g = c.geometry
        mask = mask_plane(c.nx, c.ny, g[1], g[2]) if g[0] == "plane" else mask_disk(c.nx, c.ny, g[1], g[2], g[3])
        t0 = time.perf_counter()
        t, b = bridge_history(c, mask, every=every, steps=steps, storage=storage)
        wall = time.perf_counter() - t0
        alpha = fit_exponent(t, b, b_lo, R0 / 3.0)
        row = dict(R0=R0, Rs=Rs, nu=(c.tau - 0.5) / 3.0, nx=c.nx, ny=c.ny, tau=c.tau, t_nu=c.t_nu, steps=steps,
                   every=every, alpha=alpha, t=t.tolist(), b=b.tolist(), seconds=wall)
        out.append(row)
        if log:
            log("coalescence R0=%g %dx%d tau=%.4f steps=%d alpha=%.3f (%.1f s)" % (R0, c.nx, c.ny, c.tau, steps,
                                                                                 alpha, wall))
    return out


def plane_position(rho, mask, beta, level):
    """Centre of the drop fluid (rho above level, fluid nodes) projected on the
    plane direction (cos beta, sin beta)."""
    ny, nx = rho.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    w = np.where((np.asarray(mask) == 0) & (rho > level), rho, 0.0)
    s = w.sum()
    return float(((w * xx).sum() * math.cos(beta) + (w * yy).sum() * math.sin(beta)) / s)


def sliding_study(betas, rules, *, n=400, R0=18.0, steps=6000, every=250, fit_from=2000, log=None):
    """Drop velocity along off-grid planes (Section 3.1, Fig. 2): drops of
    radius R0 in an n x n box at G = 3, rho 1.0/0.055, for each wetting rule
    and inclination, run as one batch; u_d is the least-squares slope of the
    along-plane drop position over fit_from <= t <= steps.  rules: list of
    (name, bc, params dict) for the two-component model; the single-component
    model runs as separate simulations, rules named 'sc1-...'."""
    import workloads as W

    from .sim import Simulation

    rows = []
    two = [(nm, bc, kw) for nm, bc, kw in rules if not nm.startswith("sc1")]
    one = [(nm, bc, kw) for nm, bc, kw in rules if nm.startswith("sc1")]
    t_s = np.arange(every, steps + 1, every, dtype=np.float64)
    sel = t_s >= fit_from
    if two:
        keys, cases = [], []
        for nm, bc, kw in two:
            for beta in betas:
                c = W.plane_drop(n, n, beta, R0, bc, G=3.0, rho_out=0.055, **kw)
                m = mask_plane(n, n, c.geometry[1], c.geometry[2])
                keys.append((nm, beta, c.geometry[1], m))
                cases.append((m, c.rhoA0, c.rhoB0, c.params()))
        b = Batch(cases)
        pos = np.zeros((len(keys), len(t_s)))
        try:
            for k in range(len(t_s)):
                b.step(every)
                for i, (nm, beta, brad, m) in enumerate(keys):
                    pos[i, k] = plane_position(b.fields(i, (True, False, False, False))[0], m, brad, 0.5)
                if log and (k + 1) % 8 == 0:
                    log("sliding: two-component step %d of %d" % ((k + 1) * every, steps))
        finally:
            b.close()
        for i, (nm, beta, brad, m) in enumerate(keys):
            ud = float(np.polyfit(t_s[sel], pos[i, sel], 1)[0])
            rows.append(dict(rule=nm, beta=beta, u_d=ud, pos=pos[i].tolist()))
    for nm, bc, kw in one:
        for beta in betas:
            c = W.sc1_plane_drop(n, n, beta, R0, bc, **kw)
            m = mask_plane(n, n, c.geometry[1], c.geometry[2])
            s = Simulation(m, c.rhoA0, None, **c.params())
            p = []
            try:
                for k in range(len(t_s)):
                    s.step(every)
                    p.append(plane_position(s.fields()[0], m, c.geometry[1], 0.5 * (W.SC1_RHO_L + W.SC1_RHO_V)))
            finally:
                s.close()
            p = np.array(p)
            rows.append(dict(rule=nm, beta=beta, u_d=float(np.polyfit(t_s[sel], p[sel], 1)[0]), pos=p.tolist()))
        if log:
            log("sliding: %s done" % nm)
    return rows


def main_sliding(argv):
    ap = argparse.ArgumentParser(description="Drop velocity along off-grid planes (Section 3.1).")
    ap.add_argument("--beta", default="0,10,20,30,40,45,50,60,70,80")
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--R0", type=float, default=18.0)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--fit-from", type=int, default=2000)
    ap.add_argument("--rules", default="", help="comma list of rule-name prefixes to run (default: all)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import workloads as W

    rules = [("martys-chen Gw=-0.2", W.MC, dict(Gw=-0.2)), ("martys-chen Gw=0", W.MC, dict(Gw=0.0)),
             ("llkc Gw=-0.5", W.LLKC, dict(Gw=-0.5)),
             ("improved xi=-0.2", W.IMPROVED, dict(chi=xi_to_chi(-0.2))),
             ("sc1-martys-chen Gw=-3", W.MC, dict(Gw=-3.0)), ("sc1-llkc Gw=-5", W.LLKC, dict(Gw=-5.0))]
    if a.rules:
        pre = [v.strip() for v in a.rules.split(",")]
        rules = [r for r in rules if any(r[0].startswith(p) for p in pre)]
    betas = [float(v) for v in a.beta.split(",")]
    rows = sliding_study(betas, rules, n=a.n, R0=a.R0, steps=a.steps, every=a.every, fit_from=a.fit_from,
                         log=lambda m: print(m, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(args=vars(a), rows=rows), f)
    names = [r[0] for r in rules]
    print("| rule | " + " | ".join("beta=%g" % b for b in betas) + " |")
    print("|---|" + "---|" * len(betas))
    for nm in names:
        v = {r["beta"]: r["u_d"] for r in rows if r["rule"] == nm}
        print("| %s | " % nm + " | ".join("%.1e" % v[b] for b in betas) + " |")
    return 0


def main_coalescence(argv):
    ap = argparse.ArgumentParser(description="Bridge growth of coalescing drops versus resolution (Section 4).")
    ap.add_argument("--R0", default="12.5,25,50,100,200,400")
    ap.add_argument("--Rs", type=float, default=None, help="surface radius; flat when omitted")
    ap.add_argument("--t-end", type=float, default=4.0, help="in viscous times")
    ap.add_argument("--samples", type=int, default=400)
    ap.add_argument("--nu", default="", help="comma list of viscosities at the first R0 (default: Oh = 0.286)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    nus = [float(v) for v in a.nu.split(",") if v.strip()]
    rows = coalescence_study([float(v) for v in a.R0.split(",")], a.Rs, samples=a.samples, t_end=a.t_end, nus=nus,
                             log=lambda m: print(m, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(args=vars(a), rows=rows), f)
    print("| R0 | nu | grid | tau | steps | alpha | b/R0 at t/tau_nu = 0.5, 1, 2, 4 |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        tt = np.array(r["t"]) / r["t_nu"]
        bb = np.array(r["b"]) / r["R0"]
        pts = ", ".join("%.3f" % np.interp(x, tt, bb) for x in (0.5, 1.0, 2.0, 4.0))
        print("| %g | %.3f | %dx%d | %.4f | %d | %.3f | %s |" % (r["R0"], r["nu"], r["nx"], r["ny"], r["tau"],
                                                              r["steps"], r["alpha"], pts))
    return 0


def adhesion_angles(rules, betas, *, n=400, R0=18.0, tau=1.0, G=3.0, rho_out=0.055, marks=(5000, 10000, 20000, 40000),
                    skip=3, log=None):
    """Contact angles of drops under the adhesion-force rules (Martys-Chen,
    LLKC) at the set-up of Section 3.1: box n x n, drop of radius R0 tangent to
    a plane of inclination beta, densities 1.0 / rho_out, G_AB = G,
    G_As = -G_Bs = G_w.  rules: iterable of (bc, G_w).  Returns one dict per
    (bc, G_w, beta) with the angle (half-way wall line) and the circle radius
    at each mark.  Drops at rest need beta = 0 or 45 degrees (Section 3.1)."""
    import workloads as W

    keys, cases, walls = [], [], []
    for bc, gw in rules:
        for beta in betas:
            c = W.plane_drop(n, n, beta, R0, bc, G=G, tau=tau, rho_out=rho_out, Gw=gw)
            mask = mask_plane(n, n, c.geometry[1], c.geometry[2])
            keys.append((int(bc), float(gw), float(beta)))
            cases.append((mask, c.rhoA0, c.rhoB0, c.params()))
            walls.append(wall_line(mask, range(max(1, n // 2 - int(3.5 * R0)), min(n - 1, n // 2 + int(3.5 * R0)))))
    roi = drop_roi(n, n, R0, half=4.0)
    b = Batch(cases)
    rows = [dict(bc=k[0], Gw=k[1], beta=k[2], theta=[], R=[], steps=[]) for k in keys]
    done = 0
    try:
        for m in sorted(marks):
            b.step(m - done)
            done = m
            for i, r in enumerate(rows):
                c = b.contour_fit(i, 0.5, skip, roi)
                r["theta"].append(contact_angle(c, walls[i]))
                r["R"].append(c["R"])
                r["steps"].append(m)
            if log:
                log("adhesion angles: step %d" % m)
    finally:
        b.close()
    return rows


def main_adhesion(argv):
    import workloads as W

    ap = argparse.ArgumentParser(description="Contact angles under the Martys-Chen and LLKC rules (Section 3.1).")
    ap.add_argument("--mc", default="-0.1,-0.2,-0.3,-0.4", help="G_w values of the Martys-Chen rule")
    ap.add_argument("--llkc", default="-0.3,-0.5,-0.7,-1.0", help="G_w values of the LLKC rule")
    ap.add_argument("--beta", default="0,45")
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--R0", type=float, default=18.0)
    ap.add_argument("--steps", default="5000,10000,20000,40000")
    a = ap.parse_args(argv)
    rules = [(W.MC, float(g)) for g in a.mc.split(",") if g.strip()]
    rules += [(W.LLKC, float(g)) for g in a.llkc.split(",") if g.strip()]
    betas = [float(v) for v in a.beta.split(",")]
    rows = adhesion_angles(rules, betas, n=a.n, R0=a.R0, marks=[int(v) for v in a.steps.split(",")],
                           log=lambda m: print(m, flush=True))
    print("| rule | G_w | beta | " + " | ".join("t=%d" % t for t in rows[0]["steps"]) + " |")
    print("|---|---|---|" + "---|" * len(rows[0]["steps"]))
    for r in rows:
        print("| %s | %g | %g | " % (W.BC_NAMES[r["bc"]], r["Gw"], r["beta"]) +
              " | ".join("%.1f" % t for t in r["theta"]) + " |")
    return 0


def main(argv=None):
    argv = sys.argv[1:] if argv is None else list(argv)
    if argv and argv[0] == "coalescence":
        return main_coalescence(argv[1:])
    if argv and argv[0] == "adhesion":
        return main_adhesion(argv[1:])
    if argv and argv[0] == "sliding":
        return main_sliding(argv[1:])
    if argv and argv[0] == "angles":
        argv = argv[1:]
    ap = argparse.ArgumentParser(description="Contact angle versus xi and plane inclination (improved scheme).")
    ap.add_argument("--xi", default="-0.4,-0.2,0,0.2,0.4")
    ap.add_argument("--beta", default="0,10,30,45,60")
    ap.add_argument("--avg", default="d2q25,d2q9")
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--R0", type=float, default=100.0)
    ap.add_argument("--tau", type=float, default=1.88)
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--checkpoints", type=int, default=3)
    ap.add_argument("--skip", type=int, default=3)
    ap.add_argument("--extra-skips", default="", help="comma list of further wall cuts to report")
    ap.add_argument("--out", default=None, help="write the rows as JSON here")
    a = ap.parse_args(argv)
    xis = [float(v) for v in a.xi.split(",")]
    betas = [float(v) for v in a.beta.split(",")]
    avgs = [{"d2q25": 0, "d2q9": 1}[v.strip().lower()] for v in a.avg.split(",")]

    def log(msg):
        print(msg, flush=True)

    extra = [int(v) for v in a.extra_skips.split(",") if v.strip()]
    rows = sweep(xis, betas, avgs, n=a.n, R0=a.R0, tau=a.tau, steps=a.steps, checkpoints=a.checkpoints,
                 skip=a.skip, extra_skips=extra, chunk=max(1, min(5000, a.steps // max(1, 4 * a.checkpoints))),
                 log=log)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(args=vars(a), rows=rows), f, indent=1)
    print("| avg | beta | " + " | ".join("xi=%g" % x for x in xis) + " |")
    print("|---|---|" + "---|" * len(xis))
    for avg in avgs:
        for beta in betas:
            th = [r["theta"][-1] for r in rows if r["avg"] == avg and r["beta"] == beta]
            print("| %s | %g | " % ("D2Q25" if avg == 0 else "D2Q9", beta) + " | ".join("%.1f" % t for t in th) + " |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
