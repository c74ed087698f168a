"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid problems before any device call."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "mclbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2009_12584_amd import capi

    L = capi.lib()
    declared = header_functions()
    assert len(declared) >= 30
    missing = [n for n in declared if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(declared) == sorted(capi.EXPORTS)


def _sim(**kw):
    import paper_2009_12584_amd as M

    mask = kw.pop("mask", None)
    n = kw.pop("n", 8)
    if mask is None:
        mask = np.zeros((n, n), np.uint8)
        mask[0] = mask[-1] = 1
        mask[:, 0] = mask[:, -1] = 1
    rA = kw.pop("rA", np.full(mask.shape, 0.5))
    rB = kw.pop("rB", np.full(mask.shape, 0.5))
    return M.Simulation(mask, rA, rB, **kw)


@pytest.mark.parametrize("kw,needle", [
    (dict(tau=0.5), "tau"),
    (dict(tau=float("nan")), "tau"),
    (dict(bc=4), "bc"),
    (dict(avg=2), "avg"),
    (dict(storage=7, tile_y=3), "tile_y"),
    (dict(periodic=4), "periodic"),
    (dict(G=float("inf")), "non-finite"),
    (dict(mask=np.zeros((8, 8), np.uint8)), "border"),
    (dict(rA=np.full((8, 8), -0.1)), "densities"),
    (dict(rB=np.full((8, 8), np.nan)), "densities"),
    (dict(diag_every=-1), "diag_every"),
    (dict(model=2), "model"),
    (dict(model=1, bc=2), "single-component"),
    (dict(model=1, rho0=0.0), "single-component"),
    (dict(model=0, rB=None), "rhoB0"),
    (dict(lanes=3), "lanes"),
    (dict(graph_steps=16, diag_every=6), "divide"),
    (dict(graph_steps=7, diag_every=12), "divide"),
])
def test_invalid_problems_rejected_on_host(kw, needle):
    import paper_2009_12584_amd as M

    with pytest.raises(M.LbmError) as e:
        _sim(**kw)
    assert e.value.code == -1
    assert needle in str(e.value)


def test_strerror_names_codes():
    from paper_2009_12584_amd import capi

    for code in (0, -1, -2, -3, -4, -5, -6):
        assert capi.lib().lbm_strerror(code).decode() != "unknown error"


def test_state_bytes_of_a_parameter_set():
    """The raw state is one population buffer: 9 planes of (A, B) pairs at a
    row pitch rounded up to 64 nodes, FP32; FP16 adds the FP32 rest plane."""
    from paper_2009_12584_amd.sim import state_bytes

    assert state_bytes(100, 30) == 9 * 30 * 128 * 8
    assert state_bytes(100, 30, storage="f16") == 30 * 128 * 10 * 4
    assert state_bytes(0, 30) == 0


def test_pool_footprint_counts_both_buffers():
    import paper_2009_12584_amd as M

    f32 = M.Pool.footprint(512, 256)
    f16 = M.Pool.footprint(512, 256, storage="f16")
    assert f32 >= 2 * 18 * 512 * 256 * 4
    # FP16: eight FP16 directions and the FP32 rest population per component
    assert f16 >= 2 * 2 * 512 * 256 * (8 * 2 + 4) and f16 < f32


@pytest.mark.parametrize("nx,ny,storage", [(8000, 8000, "f32"), (11000, 10000, "f16"), (16000, 16000, "f16")])
def test_grid_beyond_the_32bit_buffer_offsets_rejected(nx, ny, storage):
    """A population buffer is addressed with 32-bit byte offsets: FP32 holds 72 B
    per node, FP16 40 B (eight FP16 directions and the FP32 rest
    population of two components).  Larger grids are refused before the mask or densities are
    read, so one-element host buffers suffice here."""
    import ctypes

    from paper_2009_12584_amd import capi

    p = capi.make_params(nx, ny, storage=storage)
    mask = np.ones(1, np.uint8)
    rho = np.zeros(1)
    h = ctypes.c_void_p()
    code = capi.lib().lbm_create(ctypes.byref(p), mask.ctypes.data_as(ctypes.c_void_p),
                                 rho.ctypes.data_as(ctypes.c_void_p), rho.ctypes.data_as(ctypes.c_void_p), None,
                                 ctypes.byref(h))
    assert code == capi.LBM_EINVAL
    assert "4 GiB" in capi.lib().lbm_last_error(None).decode()
    assert not h.value


@pytest.mark.parametrize("nx,ny", [(240000, 10), (233100, 3)])
def test_grid_beyond_the_24bit_row_offsets_rejected(nx, ny):
    """Row offsets are 24-bit products (the bytes of a row of segments, at most
    72 per node, below 2^24): wider grids are refused on the host."""
    import ctypes

    from paper_2009_12584_amd import capi

    p = capi.make_params(nx, ny, storage="f16")
    mask = np.ones(1, np.uint8)
    rho = np.zeros(1)
    h = ctypes.c_void_p()
    code = capi.lib().lbm_create(ctypes.byref(p), mask.ctypes.data_as(ctypes.c_void_p),
                                 rho.ctypes.data_as(ctypes.c_void_p), rho.ctypes.data_as(ctypes.c_void_p), None,
                                 ctypes.byref(h))
    assert code == capi.LBM_EINVAL
    assert "233,000" in capi.lib().lbm_last_error(None).decode()
    assert not h.value


@pytest.mark.parametrize("storage,model,rows", [("f32", 0, 8), ("f16", 0, 16), ("f16", 1, 8), ("f32", 1, 8)])
def test_default_tile_rows_follow_storage_and_model(storage, model, rows):
    """tile_y = 0 takes 16 rows for the two-component model with FP16 storage
    and 8 otherwise.  The pool footprint counts per-tile flags and partials,
    so it equals that of the explicit default height and differs from the
    other one."""
    import ctypes

    from paper_2009_12584_amd import capi

    def footprint(ty):
        p = capi.make_params(512, 256, storage=storage, model=model, tile_y=ty)
        return int(capi.lib().lbm_pool_footprint(ctypes.byref(p)))

    other = 8 if rows == 16 else 16
    assert footprint(0) == footprint(rows) != footprint(other)
