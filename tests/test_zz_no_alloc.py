"""The allocation-free pool admission (lbm_pool_admit_noalloc) against the
allocating one (lbm_pool_admit), through the C ABI: two requests admitted in a
row through it, the second on a smaller grid, give the same fields bit for
bit as the same requests admitted the usual way, each within the FP32 bar of
the FP64 oracle; a grid whose staging exceeds the scratch array is refused
before anything is enqueued."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available()
    import paper_2009_12584_amd as M

    return M


def run_pool(M, items, noalloc_flags):
    pool = M.Pool(1 << 30, len(items))
    slots = {}
    for k, ((m, c, n), na) in enumerate(zip(items, noalloc_flags)):
        print("case: admit %dx%d %s, %d steps" % (c.nx, c.ny, "noalloc" if na else "alloc", n), flush=True)
        s = pool.admit(m, c.rhoA0, c.rhoB0, n, noalloc=na, **c.params())
        assert s is not None
        slots[s] = k
    out = {}
    for _ in range(20000):
        pool.advance(16)
        for s in pool.poll():
            out[slots[s]] = pool.fields(s)
            pool.release(s)
        if len(out) == len(items):
            break
        time.sleep(0.001)
    pool.close()
    return out


def test_noalloc_admission_matches_the_allocating_one(M, ora):
    big = W.plane_drop(420, 230, 25.0, 40.0, W.IMPROVED, G=3.0, rho_out=0.055, chi=(1.2, 0.8))
    small = W.plane_drop(150, 90, 35.0, 15.0, W.LLKC, G=3.0)
    items = []
    for c, n in ((big, 120), (small, 90)):
        m = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
        items.append((m, c, n))
    a = run_pool(M, items, (True, True))   # two calls in a row, the second smaller
    b = run_pool(M, items, (False, False))
    for k, (m, c, n) in enumerate(items):
        for x, y in zip(a[k], b[k]):
            assert np.array_equal(x, y), k
        o = ora.Oracle(m, c.rhoA0, c.rhoB0, **c.params())
        o.step(n)
        of = o.fields()
        fl = m == 0
        er = max(np.max(np.abs(a[k][0] - of[0])[fl] / of[0][fl]), np.max(np.abs(a[k][1] - of[1])[fl] / of[1][fl]))
        eu = max(np.max(np.abs(a[k][2] - of[2])[fl]), np.max(np.abs(a[k][3] - of[3])[fl]))
        print("  request %d (%dx%d): rel rho %.2e abs u %.2e" % (k, c.nx, c.ny, er, eu), flush=True)
        assert er <= 1e-5 and eu <= 1e-6


def test_noalloc_admission_refuses_a_grid_beyond_its_scratch(M):
    from paper_2009_12584_amd.capi import LBM_EINVAL, LbmError

    nx, ny = 2048, 1100  # staging of 2,252,800 nodes: 19 B each is more than 40 MiB
    m = np.zeros((ny, nx), np.uint8)
    m[0, :] = m[-1, :] = 1
    m[:, 0] = m[:, -1] = 1
    r = np.full((ny, nx), 0.5)
    pool = M.Pool(1 << 30, 2)
    with pytest.raises(LbmError) as e:
        pool.admit(m, r, r, 10, noalloc=True)
    assert e.value.code == LBM_EINVAL and "scratch" in str(e.value)
    assert pool.stats() == (0, 0)
    # the allocating admission takes it
    s = pool.admit(m, r, r, 10)
    assert s is not None
    pool.release(s)
    pool.close()
