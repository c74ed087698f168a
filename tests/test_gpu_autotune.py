"""The launch-shape autotuner on the device: it returns a shape it offers,
caches it per problem bucket, and the shape it picks gives the same fields
as any other (the kernels agree bit for bit)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_autotuner_picks_a_candidate_and_caches_it(tmp_path, monkeypatch):
    from paper_2009_12584_amd import autotune as T
    from paper_2009_12584_amd.sim import Simulation, mask_plane

    monkeypatch.setattr(T, "_CACHE_PATH", str(tmp_path / "tune.json"))
    monkeypatch.setattr(T, "_cache", None)
    c = W.plane_drop(300, 150, 30.0, 30.0, W.IMPROVED, chi=(1.2, 0.8))
    m = mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    print("case: autotune 300x150 improved", flush=True)
    cfg = T.launch_config_for(m, c.rhoA0, c.rhoB0, steps=100, **c.params())
    assert (cfg["tile_y"], cfg["lanes"]) in T.CANDIDATES
    assert (tmp_path / "tune.json").exists()
    # the cached answer comes back without timing again
    monkeypatch.setattr(T, "_time", lambda *a, **k: pytest.fail("timed again"))
    assert T.launch_config_for(m, c.rhoA0, c.rhoB0, **c.params()) == cfg
    out = []
    for shape in (cfg, dict(tile_y=4, lanes=1)):
        s = Simulation(m, c.rhoA0, c.rhoB0, **shape, **c.params())
        s.step(50)
        out.append(s.fields())
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_batch_autotuner_picks_a_candidate():
    from paper_2009_12584_amd import autotune as T
    from paper_2009_12584_amd.sim import mask_plane

    cases = W.config4_instances(4)
    items = [(mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]), c.rhoA0, c.rhoB0, c.params()) for c in cases]
    print("case: batch autotune, 4 instances", flush=True)
    cfg = T.launch_config_for_batch(items, steps=20)
    assert (cfg["tile_y"], cfg["lanes"]) in T.CANDIDATES
