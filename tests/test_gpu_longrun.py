"""GPU parity at each configuration's final step.

The GPU runs configurations 2, 3 and the 64-instance batch of configuration 4
to their full lengths (20,000, 50,000 and 10,000 steps) in the launch forms
the benchmark times (step graphs with the fused diagnostics), and is compared
with the FP64 oracle:

  - at steps 1, 10, 100 (and 1000 for configuration 2) on every fluid node,
    against the oracle run live here;
  - at 1000 and the final step of configuration 3, and the final steps of
    configuration 2 and four batch instances, on the sampled nodes of
    tests/golden/longrun_*.npz, which tests/golden/make_longrun.py wrote from
    the oracle alone (2048 random fluid nodes plus every fluid node of 24 x 24
    windows on the contact lines, the coalescence bridge and the bulk).

Bar: the FP32 one, 1e-5 relative on rho^A, rho^B and 1e-6 absolute on u.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

RHO_TOL = 1e-5
U_TOL = 1e-6


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available()
    import paper_2009_12584_amd as M

    return M


def golden(name, case, mask):
    import make_longrun

    g = np.load(os.path.join(HERE, "golden", "longrun_%s.npz" % name), allow_pickle=False)
    assert str(g["input_sha"]) == make_longrun.input_hash(case, mask), "stale golden file for %s" % name
    return g


def full_errors(mask, gf, of):
    fl = mask == 0
    er = max(np.max(np.abs(gf[0] - of[0])[fl] / of[0][fl]), np.max(np.abs(gf[1] - of[1])[fl] / of[1][fl]))
    eu = max(np.max(np.abs(gf[2] - of[2])[fl]), np.max(np.abs(gf[3] - of[3])[fl]))
    return er, eu


def sampled_errors(g, T, gf):
    idx = g["idx"]
    got = [f.ravel()[idx] for f in gf]
    ref = [g["%s_%d" % (k, T)].astype(np.float64) for k in ("rhoA", "rhoB", "ux", "uy")]
    er = max(np.max(np.abs(got[0] - ref[0]) / ref[0]), np.max(np.abs(got[1] - ref[1]) / ref[1]))
    eu = max(np.max(np.abs(got[2] - ref[2])), np.max(np.abs(got[3] - ref[3])))
    return er, eu


def check(label, T, er, eu, n=None):
    say("  %s t=%d: max rel rho %.3e, max abs u %.3e%s" % (label, T, er, eu, "" if n is None else " (%d nodes)" % n))
    assert er <= RHO_TOL and eu <= U_TOL, (label, T, er, eu)


@pytest.mark.parametrize("ty,lanes", [(8, 2), (8, 1)], ids=["two-lane-64x8", "one-lane-64x8"])
def test_config2_to_20000_steps(M, ora, ty, lanes):
    c = W.config2()
    mask = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    g = golden("c2", c, mask)
    say("case: config 2, %d steps, graphs of 100 with diagnostics, tile rows %d, lanes %d" % (c.steps, ty, lanes))
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0, tile_y=ty, lanes=lanes, graph_steps=100, diag_every=100,
                       drift_tol=1e-4, **c.params())
    o = ora.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    for T in (1, 10, 100, 1000):
        sim.step(T - sim.t)
        o.step(T - o.t)
        check("config 2 (all fluid nodes)", T, *full_errors(mask, sim.fields(), o.fields()))
    sim.step(c.steps - sim.t)
    check("config 2 (sampled)", c.steps, *sampled_errors(g, c.steps, sim.fields()), n=g["idx"].size)
    d = sim.diag()
    assert d["flags"] == 0
    say("  mass drift after %d steps: %.2e, %.2e" % (c.steps, *(abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k]
                                                                 for k in range(2))))
    assert sim.launch_counts()["graph_steps"] >= c.steps - 1000
    sim.close()


def test_config3_to_50000_steps(M, ora):
    c = W.config3(0)
    gm = c.geometry
    mask = M.mask_disk(c.nx, c.ny, gm[1], gm[2], gm[3])
    g = golden("c3", c, mask)
    say("case: config 3 (seed 0), %d steps, graphs of 100 with diagnostics" % c.steps)
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0, graph_steps=100, diag_every=100, drift_tol=1e-4, **c.params())
    o = ora.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    for T in (1, 10, 100):
        sim.step(T - sim.t)
        o.step(T - o.t)
        check("config 3 (all fluid nodes)", T, *full_errors(mask, sim.fields(), o.fields()))
    del o
    for T in (1000, c.steps):
        sim.step(T - sim.t)
        check("config 3 (sampled)", T, *sampled_errors(g, T, sim.fields()), n=g["idx"].size)
    d = sim.diag()
    assert d["flags"] == 0
    say("  mass drift after %d steps: %.2e, %.2e" % (c.steps, *(abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k]
                                                                 for k in range(2))))
    sim.close()


def test_config4_batch_to_10000_steps(M, ora):
    cases = W.config4_instances(64)
    masks = [M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]
    picks = (0, 3, 5, 29)
    goldens = {k: golden("c4-%02d" % k, cases[k], masks[k]) for k in picks}
    say("case: batch of 64 instances, 10000 steps, graphs of 100 with diagnostics every 100")
    b = M.Batch([(m, c.rhoA0, c.rhoB0, dict(c.params(), diag_every=100, drift_tol=1e-4))
                 for m, c in zip(masks, cases)], graph_steps=100)
    try:
        oras = {k: ora.Oracle(masks[k], cases[k].rhoA0, cases[k].rhoB0, **cases[k].params()) for k in picks}
        t = 0
        for T in (1, 10, 100):
            b.step(T - t)
            t = T
            for k in picks:
                oras[k].step(T - oras[k].t)
                check("instance %d %s (all fluid nodes)" % (k, cases[k].name), T,
                      *full_errors(masks[k], b.fields(k), oras[k].fields()))
        oras.clear()
        T = cases[0].steps
        b.step(T - t)
        for k in picks:
            check("instance %d %s (sampled)" % (k, cases[k].name), T, *sampled_errors(goldens[k], T, b.fields(k)),
                  n=goldens[k]["idx"].size)
        for k in range(64):
            assert b.diag(k)["flags"] == 0, k
        say("  launches:", b.launch_counts())
    finally:
        b.close()
