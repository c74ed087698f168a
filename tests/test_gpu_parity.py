"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar (FP32 storage): max over fluid nodes of |rho_gpu - rho_ora| / rho_ora <= 1e-5
and |u_gpu - u_ora| <= 1e-6; wall masks and stair classification bit-exact.
"""
import math
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-5
U_TOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2009_12584_amd as M

    return M


def gpu_mask(M, c):
    if c.mask_user is not None:
        return c.mask_user
    g = c.geometry
    if g[0] == "plane":
        return M.mask_plane(c.nx, c.ny, g[1], g[2])
    if g[0] == "disk":
        return M.mask_disk(c.nx, c.ny, g[1], g[2], g[3])
    raise ValueError(g)


def ora_mask(ora, c):
    if c.mask_user is not None:
        return c.mask_user
    g = c.geometry
    if g[0] == "plane":
        return ora.mask_plane(c.nx, c.ny, g[1], g[2])
    return ora.mask_disk(c.nx, c.ny, g[1], g[2], g[3])


def errors(mask, gf, of):
    fl = mask == 0
    ga, gb, gux, guy = gf
    oa, ob, oux, ouy = of
    er = max(np.max(np.abs(ga - oa)[fl] / oa[fl]), np.max(np.abs(gb - ob)[fl] / ob[fl]))
    eu = max(np.max(np.abs(gux - oux)[fl]), np.max(np.abs(guy - ouy)[fl]))
    return er, eu


def compare_run(M, ora, c, checkpoints, **extra):
    say("case", c.name, c.nx, c.ny, "bc", c.bc, "checkpoints", checkpoints, extra)
    mask = gpu_mask(M, c)
    assert np.array_equal(mask, ora_mask(ora, c)), "wall mask differs"
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0, **c.params(), **extra)
    o = ora.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    out = []
    for T in checkpoints:
        sim.step(T - sim.t)
        o.step(T - o.t)
        er, eu = errors(mask, sim.fields(), o.fields())
        say("  t=%d rel rho %.3e abs u %.3e" % (T, er, eu))
        out.append((T, er, eu))
    sim.close()
    return out


# ------------------------------------------------------------ geometry

@pytest.mark.parametrize("nx,ny,beta_deg,R0", [(64, 64, 0.0, 15.0), (512, 256, 30.0, 40.0), (400, 400, 70.0, 18.0),
                                               (333, 121, 17.3, 20.0), (1000, 1000, 45.0, 100.0),
                                               (5600, 4000, 30.0, 400.0)])
def test_plane_mask_bit_exact(gpu, ora, nx, ny, beta_deg, R0):
    b = math.radians(beta_deg)
    assert np.array_equal(gpu.mask_plane(nx, ny, b, R0), ora.mask_plane(nx, ny, b, R0))
    assert np.array_equal(gpu.mask_plane(nx, ny, b, R0, borders=False),
                          ora.mask_plane(nx, ny, b, R0, borders=False))


def test_disk_mask_bit_exact(gpu, ora):
    c = W.config3(0)
    g = c.geometry
    assert np.array_equal(gpu.mask_disk(c.nx, c.ny, g[1], g[2], g[3]), ora.mask_disk(c.nx, c.ny, g[1], g[2], g[3]))
    assert np.array_equal(gpu.mask_disk(301, 257, 150.5, 100.25, 77.7), ora.mask_disk(301, 257, 150.5, 100.25, 77.7))


@pytest.mark.parametrize("which", ["c1", "c2", "c3", "periodic-xy"])
def test_classification_bit_exact(gpu, ora, which):
    if which == "c1":
        c = W.config1()
    elif which == "c2":
        c = W.config2()
    elif which == "c3":
        c = W.config3(1)
    else:
        rng = np.random.default_rng(5)
        m = (rng.random((70, 130)) < 0.2).astype(np.uint8)
        c = W.Case("rand", 130, 70, periodic=3, rhoA0=np.full((70, 130), 0.5), rhoB0=np.full((70, 130), 0.5),
                   mask_user=m)
    mask = gpu_mask(gpu, c)
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, **c.params())
    nbr, cls = sim.classify()
    sim.close()
    onbr, ocls = ora.classify(mask, c.periodic)
    assert np.array_equal(nbr, onbr) and np.array_equal(cls, ocls)


# ------------------------------------------------------ step-0 quantities

@pytest.mark.parametrize("bc", [W.MC, W.LLKC, W.IMPROVED, W.FIXED])
@pytest.mark.parametrize("avg", [0, 1])
def test_forces_and_virtual_density_at_step0(gpu, ora, bc, avg):
    if bc != W.IMPROVED and avg == 1:
        pytest.skip("averaging lattice only matters for the improved scheme")
    c = W.plane_drop(203, 97, 25.0, 15.0, bc, G=3.0, chi=(1.2, 0.8))
    c.avg = avg
    rA, rB = W.random_mixture(c.nx, c.ny, seed=9, mean=0.5, amp=0.3)
    mask = gpu_mask(gpu, c)
    sim = gpu.Simulation(mask, rA, rB, **c.params())
    o = ora.Oracle(mask, rA, rB, **c.params())
    g = sim.forces()
    f = o.forces() + o.virtual_density()
    sim.close()
    scale = max(np.abs(x).max() for x in f[:4])
    for k in range(4):
        assert np.max(np.abs(g[k] - f[k])) <= 2e-6 * scale, k
    for k in (4, 5):
        assert np.max(np.abs(g[k] - f[k])) <= 1e-6 * max(1.0, np.abs(f[k]).max()), k


# ------------------------------------------------------------ dynamics

@pytest.mark.parametrize("bc,avg,chi", [(W.MC, 0, (1.0, 1.0)), (W.LLKC, 0, (1.0, 1.0)), (W.IMPROVED, 0, (1.0, 1.0)),
                                        (W.IMPROVED, 1, (1.15, 0.85)), (W.FIXED, 0, (0.7, 0.3))],
                         ids=["martys-chen", "llkc", "improved-d2q25", "improved-d2q9", "fixed-virtual"])
def test_parity_ragged_tiles_all_bcs(gpu, ora, bc, avg, chi):
    """Several tiles with ragged right/bottom edges, G = 3 demixing, every rule."""
    c = W.plane_drop(203, 97, 25.0, 15.0, bc, G=3.0, rho_out=0.055, chi=chi)
    c.avg = avg
    for T, er, eu in compare_run(gpu, ora, c, [1, 10, 100, 300]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


@pytest.mark.parametrize("periodic", [1, 2, 3])
def test_parity_periodic_wrap(gpu, ora, periodic):
    nx, ny = 130, 37
    m = np.zeros((ny, nx), np.uint8)
    if not periodic & 1:
        m[:, 0] = m[:, -1] = 1
    if not periodic & 2:
        m[0, :] = m[-1, :] = 1
    m[10:20, 40:47] = 1  # an obstacle
    rA, rB = W.random_mixture(nx, ny, seed=periodic, amp=0.1)
    c = W.Case("periodic%d" % periodic, nx, ny, periodic=periodic, tau=0.8, G=2.5, bc=W.IMPROVED, chiA=1.1,
               chiB=0.9, rhoA0=rA, rhoB0=rB, mask_user=m)
    for T, er, eu in compare_run(gpu, ora, c, [1, 50, 200]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


@pytest.mark.parametrize("nx,ny,periodic,ty", [(130, 33, 2, 32), (65, 40, 3, 8), (67, 37, 3, 16)],
                         ids=["y33-tile32", "x65-tile8", "x67-tile16"])
def test_parity_periodic_size_just_above_a_tile(gpu, ora, nx, ny, periodic, ty):
    """A periodic size just above one tile: the last tile's rows (or columns)
    beyond the lattice and its 4-node reach wrap past the far side, which the
    compare-and-add wrap cannot map back (33 rows in 32-row tiles reach row 67);
    such sizes must take the modulo wrap.  Improved scheme with an obstacle, so
    the 3-node density frame is in use."""
    m = np.zeros((ny, nx), np.uint8)
    if not periodic & 1:
        m[:, 0] = m[:, -1] = 1
    if not periodic & 2:
        m[0, :] = m[-1, :] = 1
    m[10:18, 30:37] = 1
    rA, rB = W.random_mixture(nx, ny, seed=11, amp=0.1)
    c = W.Case("wrap-%dx%d" % (nx, ny), nx, ny, periodic=periodic, tau=0.8, G=2.5, bc=W.IMPROVED, chiA=1.1,
               chiB=0.9, rhoA0=rA, rhoB0=rB, mask_user=m)
    for T, er, eu in compare_run(gpu, ora, c, [1, 30, 120], tile_y=ty):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


def test_parity_tiny_periodic_box_smaller_than_tile(gpu, ora):
    nx, ny = 5, 3
    rA, rB = W.random_mixture(nx, ny, seed=2, amp=0.2)
    c = W.Case("tiny", nx, ny, periodic=3, G=2.0, bc=W.MC, rhoA0=rA, rhoB0=rB, mask_user=np.zeros((ny, nx), np.uint8))
    for T, er, eu in compare_run(gpu, ora, c, [1, 7, 60]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


def test_parity_config1_full(gpu, ora):
    """64x64, periodic x, flat walls, Martys-Chen, 2000 steps (the oracle in FP64)."""
    c = W.config1()
    for T, er, eu in compare_run(gpu, ora, c, [1, 10, 100, 1000, 2000]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


@pytest.mark.parametrize("ty,lanes", [(8, 2), (4, 1)], ids=["two-lane-64x8", "one-lane-64x4"])
def test_parity_config2_full_size(gpu, ora, ty, lanes):
    """512x256 30-degree stair, improved scheme, at the size the bench times and
    in the launch shapes its autotuner picks between."""
    c = W.config2()
    for T, er, eu in compare_run(gpu, ora, c, [1, 10, 200], tile_y=ty, lanes=lanes):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


def test_parity_config3_full_size(gpu, ora):
    """1024 x 1024, disk R = 300 with two drops on it, improved scheme with
    chi^A != chi^B, at full size for 200 steps."""
    c = W.config3(2)
    for T, er, eu in compare_run(gpu, ora, c, [1, 10, 200]):
        assert er <= RHO_TOL and eu <= U_TOL, (T, er, eu)


# ------------------------------------------------- determinism and invariants

@pytest.mark.parametrize("bc", [W.MC, W.LLKC, W.IMPROVED])
def test_tile_shapes_and_lanes_bit_identical_and_runs_repeat(gpu, ora, bc):
    """Every tile height, one or two lanes per node: the same bits."""
    c = W.plane_drop(300, 150, 33.0, 20.0, bc, G=3.0, chi=(1.1, 0.9))
    mask = gpu_mask(gpu, c)
    res = []
    for ty, lanes in ((4, 1), (8, 1), (16, 1), (32, 1), (4, 2), (8, 2), (16, 2), (32, 2), (8, 1)):
        say("case: tile rows %d lanes %d" % (ty, lanes))
        sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, tile_y=ty, lanes=lanes, **c.params())
        sim.step(150)
        res.append(sim.fields())
        sim.close()
    for r in res[1:]:
        for a, b in zip(res[0], r):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("bc", [W.MC, W.LLKC, W.IMPROVED])
def test_fp16_tile_shapes_and_lanes_bit_identical(gpu, ora, bc):
    """FP16 storage, every tile height, one or two lanes per node: the same
    bits.  The one-lane step reads the stored FP16 halves straight into
    mixed-precision adds, subtracts and multiply-adds; the two-lane step
    converts them to FP32 first.  Equal bits pin the mixed sums and
    differences to the plain FP32 arithmetic, and both round the stored
    populations once to FP16."""
    c = W.plane_drop(300, 150, 33.0, 20.0, bc, G=3.0, chi=(1.1, 0.9))
    mask = gpu_mask(gpu, c)
    res = []
    for ty, lanes in ((8, 1), (4, 1), (16, 1), (32, 1), (8, 2), (4, 2), (32, 2)):
        say("case: FP16, tile rows %d lanes %d" % (ty, lanes))
        sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, storage="f16", tile_y=ty, lanes=lanes, **c.params())
        sim.step(150)
        res.append(tuple(sim.fields()) + (sim.get_state()[0],))
        sim.close()
    for r in res[1:]:
        for a, b in zip(res[0], r):
            assert np.array_equal(a, b)


def test_graph_replay_matches_plain_launches(gpu, ora):
    c = W.plane_drop(256, 128, 30.0, 20.0, W.IMPROVED, G=3.0)
    mask = gpu_mask(gpu, c)
    a = gpu.Simulation(mask, c.rhoA0, c.rhoB0, **c.params())
    b = gpu.Simulation(mask, c.rhoA0, c.rhoB0, graph_steps=16, diag_every=1, lanes=2, **c.params())
    # graphs replay from multiples of 16 only, plain launches in between:
    # 1 plain; 15 plain, 16 graph, 9 plain; 7, 16, 10; 6, 48, 10
    for n in (1, 40, 33, 64):
        a.step(n)
        b.step(n)
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)
    assert b.launch_counts() == {"graph_steps": 80, "plain_steps": 58}
    assert a.launch_counts() == {"graph_steps": 0, "plain_steps": 138}
    a.close()
    b.close()


def test_numeric_flags_raised_from_a_host_made_state(gpu, ora):
    """Failure handling, forced from the host: a state whose deviations were
    scaled (mass no longer that of step 0) raises the drift flag, a state of
    NaNs the non-finite flag; lbm_diag then returns LBM_ENUMERIC.  The kernels
    run normally on both (NaN arithmetic does not fault)."""
    from paper_2009_12584_amd.capi import LBM_ENUMERIC, LbmError

    c = W.plane_drop(160, 80, 20.0, 12.0, W.MC, G=3.0)
    mask = gpu_mask(gpu, c)
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, diag_every=10, drift_tol=1e-6, **c.params())
    sim.step(20)
    assert sim.diag()["flags"] == 0
    st, t = sim.get_state()
    scaled = st.view(np.float32) * np.float32(1.5)
    sim.set_state(scaled.view(np.uint8), t)
    sim.step(10)
    with pytest.raises(LbmError) as e:
        sim.diag()
    assert e.value.code == LBM_ENUMERIC
    d = sim.diag(raise_on_flags=False)
    assert d["flags"] & 4 and not d["flags"] & 1
    # a flagged simulation refuses to step on
    with pytest.raises(LbmError) as e:
        sim.step(1)
    assert e.value.code == LBM_ENUMERIC
    sim.close()
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, diag_every=10, drift_tol=1e-6, **c.params())
    nan = np.full(st.size // 4, np.nan, np.float32)
    sim.set_state(nan.view(np.uint8), t)
    sim.step(10)
    d = sim.diag(raise_on_flags=False)
    assert d["flags"] & 1
    sim.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_checkpoint_resume_bit_exact(gpu, ora, storage):
    """The state copy holds the whole population buffer (with FP16 storage, the
    FP32 rest-population plane too): a resumed run is bit-identical."""
    c = W.plane_drop(200, 100, 30.0, 15.0, W.LLKC, G=3.0)
    mask = gpu_mask(gpu, c)
    a = gpu.Simulation(mask, c.rhoA0, c.rhoB0, storage=storage, **c.params())
    a.step(37)
    st, t = a.get_state()
    a.step(50)
    ref = a.fields()
    b = gpu.Simulation(mask, c.rhoA0, c.rhoB0, storage=storage, **c.params())
    b.set_state(st, t)
    b.step(50)
    for x, y in zip(ref, b.fields()):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_diagnostics_match_oracle_totals(gpu, ora):
    c = W.plane_drop(203, 97, 25.0, 15.0, W.IMPROVED, G=3.0)
    mask = gpu_mask(gpu, c)
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, diag_every=10, drift_tol=1e-5, **c.params())
    o = ora.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    sim.step(200)
    o.step(200)
    d = sim.diag()
    t = o.totals()
    assert d["step"] == 200 and d["flags"] == 0
    assert d["mass"][0] == pytest.approx(t[0], rel=1e-6)
    assert d["mass"][1] == pytest.approx(t[1], rel=1e-6)
    assert d["mass0"][0] == pytest.approx(t[0], rel=1e-6)
    assert abs(d["momentum"][0] - t[2]) < 1e-6 * t[1]
    assert abs(d["momentum"][1] - t[3]) < 1e-6 * t[1]
    _, _, ux, uy = o.fields()
    assert d["max_speed"] == pytest.approx(np.sqrt(ux ** 2 + uy ** 2).max(), rel=1e-4)
    sim.close()


def test_mass_conserved_config2_20k_steps(gpu, ora):
    """Property at full size and full length: per-component mass stays at step 0's
    value (FP32 storage, FP64 reduction) and the drift flag stays clear."""
    c = W.config2()
    mask = gpu_mask(gpu, c)
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, diag_every=1000, drift_tol=1e-4, **c.params())
    sim.step(c.steps)
    d = sim.diag()
    for k in range(2):
        assert abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k] < 2e-5
    sim.close()


def test_fp16_mass_conserved_config2_20k_steps(gpu, ora):
    """FP16 storage keeps the rest population, which takes each node's exact mass
    remainder, in FP32: the node's mass then moves by one FP32 rounding per step
    as with FP32 storage, and the same bound holds.  (With the remainder rounded
    to FP16 this case lost 4% of a component's mass.)"""
    c = W.config2()
    mask = gpu_mask(gpu, c)
    print("case: config 2, FP16 storage, %d steps" % c.steps, flush=True)
    sim = gpu.Simulation(mask, c.rhoA0, c.rhoB0, diag_every=1000, drift_tol=1e-4, storage="f16", **c.params())
    sim.step(c.steps)
    d = sim.diag()
    say("fp16 mass drift", [abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k] for k in range(2)])
    assert d["flags"] == 0
    for k in range(2):
        assert abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k] < 2e-5
    sim.close()


def test_fp16_storage_error_is_the_storage_models(gpu, ora):
    """FP16 deviation storage against the FP64 oracle, held to twice the error
    of the oracle with the same storage rounding applied after every step
    (oracle/storage_model.py): the FP16 path may add no error of its own
    beyond the format's."""
    from oracle.storage_model import StorageModel

    c = W.plane_drop(203, 97, 25.0, 15.0, W.IMPROVED)
    res = compare_run(gpu, ora, c, [10, 100], storage="f16")
    mask = ora_mask(ora, c)
    exact = ora.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
    model = StorageModel(mask, c.rhoA0, c.rhoB0, **c.params())
    for T, er, eu in res:
        exact.step(T - exact.t)
        model.step(T - model.t)
        mr, mu = errors(mask, model.fields(), exact.fields())
        say("  t=%d fp16 %.3e %.3e, storage model %.3e %.3e" % (T, er, eu, mr, mu))
        assert er < 2 * mr and eu < 2 * mu
        assert er < 5e-3 and eu < 1e-3
