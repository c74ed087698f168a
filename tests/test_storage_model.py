"""Pins of the FP16 storage model (oracle/storage_model.py), the oracle-side
model of the library's FP16 population storage from which the FP16 tolerance
is derived.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.storage_model import (FP16_SCALE, StorageModel, default_rho_ref, from_origin, origin_maps,
                                  round_fp16_storage, to_origin)


def plane_case(nx=70, ny=44, beta=20.0, R0=9.0, bc=W.MC):
    c = W.plane_drop(nx, ny, beta, R0, bc)
    m = oracle.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    return c, m


def random_state(rng, mask, lo=0.01, hi=0.2):
    ny, nx = mask.shape
    F = rng.uniform(lo, hi, size=(2, 9, ny * nx))
    F[:, :, mask.ravel() != 0] = 0.0
    return F


@pytest.mark.parametrize("periodic", [0, 1, 3])
def test_origin_maps_are_the_oracles_streaming(periodic):
    """With no collision (tau -> infinity) and no force (G = 0, G_w = 0) an
    oracle step is streaming with half-way bounce-back alone: it must move an
    arbitrary state exactly as from_origin does."""
    rng = np.random.default_rng(4)
    if periodic == 3:
        mask = np.zeros((23, 31), np.uint8)
        mask[8:13, 10:17] = 1  # an obstacle
    elif periodic == 1:
        mask = np.zeros((20, 33), np.uint8)
        mask[0, :] = mask[-1, :] = 1
        mask[1:6, 12] = 1
    else:
        _, mask = plane_case()
    ny, nx = mask.shape
    rho = np.full((ny, nx), 0.5)
    o = oracle.Oracle(mask, rho, rho, tau=1e9, G=0.0, bc=W.MC, Gw=0.0, periodic=periodic)
    F = random_state(rng, mask)
    o.set_populations(F.reshape(2, 9, ny, nx))
    o.step(1)
    got = o.populations().reshape(2, 9, -1)
    want = from_origin(F, origin_maps(mask, periodic))
    fl = mask.ravel() == 0
    assert np.max(np.abs(got[:, :, fl] - want[:, :, fl])) < 1e-8


def test_origin_maps_are_a_bijection_on_fluid_nodes():
    c, m = plane_case()
    maps = origin_maps(m, 0)
    hits = np.zeros((9, m.size), int)
    for dest, src, sdir in maps:
        np.add.at(hits, (sdir, src), 1)
    fl = m.ravel() == 0
    assert np.all(hits[:, fl] == 1) and np.all(hits[:, ~fl] == 0)
    Q = random_state(np.random.default_rng(1), m)
    assert np.array_equal(to_origin(from_origin(Q, maps), maps)[:, :, fl], Q[:, :, fl])


def test_fp16_rounding_keeps_each_nodes_mass_and_rounds_to_nearest():
    rng = np.random.default_rng(2)
    c, m = plane_case()
    fl = m.ravel() == 0
    w = oracle.lattice()["w9"]
    rho_ref = (0.03, 0.05)
    Q = np.zeros((2, 9, m.size))
    for k in range(2):
        rho = rng.uniform(0.03, 1.0, size=m.size)
        Q[k] = w[:, None] * rho[None, :] * (1 + 0.01 * rng.standard_normal((9, m.size)))
    R = round_fp16_storage(Q, fl, rho_ref)
    for k in range(2):
        mass_in, mass_out = Q[k][:, fl].sum(0), R[k][:, fl].sum(0)
        # one FP32 rounding of the rest deviation
        assert np.max(np.abs(mass_out - mass_in) / mass_in) < 2e-7
        dev = Q[k][1:, fl] - w[1:, None] * rho_ref[k]
        kept = R[k][1:, fl] - w[1:, None] * rho_ref[k]
        # half an FP16 unit in the last place (2^-11 relative), plus the
        # subnormal spacing 2^-24 / scale
        assert np.all(np.abs(kept - dev) <= np.abs(dev) * 2.0 ** -11 + 2.0 ** -25 / FP16_SCALE + 1e-15)
        # and what IEEE round-to-nearest gives on the scaled value (up to the
        # FP64 rounding of adding and removing w_i rho_ref)
        nearest = (dev * FP16_SCALE).astype(np.float16).astype(np.float64)
        assert np.max(np.abs(kept * FP16_SCALE - nearest)) < 1e-11
    # values already on the FP16 grid are kept exactly
    R2 = round_fp16_storage(R, fl, rho_ref)
    assert np.max(np.abs(R2[:, 1:] - R[:, 1:])) == 0.0


def test_uniform_mixture_at_rest_is_a_fixed_point_of_the_model():
    m = np.zeros((16, 24), np.uint8)
    rA = np.full(m.shape, 0.6)
    rB = np.full(m.shape, 0.4)
    s = StorageModel(m, rA, rB, tau=1.0, G=0.9, bc=W.MC, Gw=0.0, periodic=3)
    s.step(30)
    f = s.fields()
    assert np.max(np.abs(f[0] - 0.6)) < 1e-12 and np.max(np.abs(f[2])) < 1e-12


def test_model_conserves_mass_and_its_error_is_the_storage_rounding():
    c, m = plane_case()
    prm = c.params()
    exact = oracle.Oracle(m, c.rhoA0, c.rhoB0, **prm)
    s = StorageModel(m, c.rhoA0, c.rhoB0, **prm)
    assert s.rho_ref == default_rho_ref(m, c.rhoA0, c.rhoB0)
    t0 = s.totals()
    exact.step(100)
    s.step(100)
    t1 = s.totals()
    for k in range(2):
        assert abs(t1[k] - t0[k]) / t0[k] < 1e-8
    got, ref = s.fields(), exact.fields()
    fl = m == 0
    er = max(np.max(np.abs(got[k] - ref[k])[fl] / ref[k][fl]) for k in (0, 1))
    # FP16 storage perturbs the run far above FP64 rounding and far below the
    # densities themselves
    assert 1e-5 < er < 1e-2
