"""GPU parity of the single-component multiphase model against the FP64 oracle.

Same bar as the two-component path (FP32 storage): max over fluid nodes of
|rho_gpu - rho_ora| / rho_ora <= 1e-5 and |u_gpu - u_ora| <= 1e-6.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5
U_TOL = 1e-6


def _run(ora, c, mask, checkpoints, **extra):
    from paper_2009_12584_amd.sim import Simulation

    print("case", c.name, c.nx, c.ny, "bc", c.bc, "checkpoints", checkpoints, extra, flush=True)
    sim = Simulation(mask, c.rhoA0, None, **c.params(), **extra)
    o = ora.Oracle(mask, c.rhoA0, None, **c.params())
    fl = mask == 0
    out = []
    for T in checkpoints:
        sim.step(T - sim.t)
        o.step(T - o.t)
        g, r = sim.fields(), o.fields()
        er = np.max(np.abs(g[0] - r[0])[fl] / r[0][fl])
        eu = max(np.max(np.abs(g[2] - r[2])[fl]), np.max(np.abs(g[3] - r[3])[fl]))
        assert np.all(g[1] == 0.0)
        print("  t=%d rel rho %.3e abs u %.3e" % (T, er, eu), flush=True)
        out.append((T, er, eu))
    sim.close()
    return out


@pytest.mark.parametrize("bc", [W.MC, W.LLKC], ids=["martys-chen", "llkc"])
def test_sc1_parity_ragged_tiles(ora, bc):
    from paper_2009_12584_amd.sim import mask_plane

    c = W.sc1_plane_drop(203, 97, 25.0, 15.0, bc)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    assert np.array_equal(m, ora.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]))
    for T, er, eu in _run(ora, c, m, [1, 10, 100, 300]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


@pytest.mark.parametrize("ty", [4, 16])
def test_sc1_parity_periodic_and_tile_shapes(ora, ty):
    """A drop across both periodic borders (a spinodal start would amplify the
    FP32/FP64 rounding difference exponentially and is left out)."""
    nx, ny = 101, 96
    yy, xx = np.mgrid[0:ny, 0:nx]
    dx = np.minimum(np.abs(xx - 5), nx - np.abs(xx - 5))
    dy = np.minimum(np.abs(yy - 90), ny - np.abs(yy - 90))
    rA = np.where(dx ** 2 + dy ** 2 <= 20 ** 2, W.SC1_RHO_L, W.SC1_RHO_V).astype(np.float64)
    c = W.Case("sc1-periodic-drop", nx, ny, periodic=3, tau=0.9, G=W.SC1_G, bc=W.MC, Gw=0.0, rhoA0=rA, model=1)
    m = np.zeros((ny, nx), np.uint8)
    for T, er, eu in _run(ora, c, m, [1, 50, 400], tile_y=ty):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


def test_sc1_forces_at_step0_and_mass_diag(ora):
    from paper_2009_12584_amd.sim import Simulation, mask_plane

    c = W.sc1_plane_drop(150, 90, 30.0, 14.0, W.LLKC)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    print("case: sc1 forces at step 0 and FP64 mass", flush=True)
    s = Simulation(m, c.rhoA0, None, diag_every=50, **c.params())
    o = ora.Oracle(m, c.rhoA0, None, **c.params())
    g = s.forces()
    f = o.forces()
    scale = max(np.abs(f[0]).max(), np.abs(f[1]).max())
    assert np.max(np.abs(g[0] - f[0])) <= 2e-6 * scale and np.max(np.abs(g[1] - f[1])) <= 2e-6 * scale
    assert np.all(g[2] == 0) and np.all(g[3] == 0)
    s.step(500)
    d = s.diag()
    assert d["mass"][1] == 0.0
    assert abs(d["mass"][0] - d["mass0"][0]) / d["mass0"][0] < 1e-6
    o.step(500)
    assert d["mass"][0] == pytest.approx(o.totals()[0], rel=1e-6)
    s.close()


def test_sc1_fp16_storage_error_is_reported_and_small(ora):
    from paper_2009_12584_amd.sim import Simulation, mask_plane

    c = W.sc1_plane_drop(160, 120, 30.0, 16.0, W.MC)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    print("case: sc1 fp16 vs fp32, 500 steps", flush=True)
    a = Simulation(m, c.rhoA0, None, storage="f32", **c.params())
    b = Simulation(m, c.rhoA0, None, storage="f16", **c.params())
    a.step(500)
    b.step(500)
    ra, rb = a.fields()[0], b.fields()[0]
    fl = m == 0
    err = np.max(np.abs(ra - rb)[fl] / ra[fl])
    print("  fp16 vs fp32 max rel rho %.3e" % err, flush=True)
    assert err < 5e-2
    a.close()
    b.close()


def test_sc1_fp16_mass_conserved(ora):
    """The rest population stays FP32 under FP16 storage: mass drift as in FP32."""
    from paper_2009_12584_amd.sim import Simulation, mask_plane

    c = W.sc1_plane_drop(512, 256, 30.0, 40.0, W.MC)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    print("case: sc1 fp16 mass, 512x256, 10000 steps", flush=True)
    s = Simulation(m, c.rhoA0, None, storage="f16", diag_every=1000, **c.params())
    s.step(10000)
    d = s.diag()
    drift = abs(d["mass"][0] - d["mass0"][0]) / d["mass0"][0]
    print("  fp16 mass drift %.3e" % drift, flush=True)
    assert drift < 2e-5
    s.close()


def test_batch_and_pool_reject_the_single_component_model(ora):
    from paper_2009_12584_amd.capi import LBM_EINVAL, LbmError
    from paper_2009_12584_amd.sim import Batch, Pool, mask_plane

    c = W.sc1_plane_drop(80, 60, 0.0, 10.0, W.MC)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    with pytest.raises(LbmError) as e:
        Batch([(m, c.rhoA0, c.rhoA0, c.params())])
    assert e.value.code == LBM_EINVAL
    p = Pool(1 << 26, 2)
    with pytest.raises(LbmError) as e:
        p.admit(m, c.rhoA0, c.rhoA0, 10, **c.params())
    assert e.value.code == LBM_EINVAL
    p.close()


def test_sc1_graph_replay_and_diagnostics_do_not_change_results(ora):
    """Plain launches, captured graphs and the fused FP64 diagnostics give the
    same bits (no contraction differences between kernel variants)."""
    from paper_2009_12584_amd.sim import Simulation, mask_plane

    c = W.sc1_plane_drop(180, 100, 30.0, 15.0, W.LLKC)
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    print("case: sc1 graph and diag variants", flush=True)
    a = Simulation(m, c.rhoA0, None, **c.params())
    b = Simulation(m, c.rhoA0, None, graph_steps=16, diag_every=1, **c.params())
    for n in (1, 40, 33, 64):
        a.step(n)
        b.step(n)
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)
    a.close()
    b.close()
