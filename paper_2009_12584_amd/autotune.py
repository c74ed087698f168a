"""Launch-shape autotuner for the step kernels.

A tile is 64 nodes wide (one wavefront row) and TY rows tall, TY in
{4, 8, 16, 32}; the two-component step runs with one lane per node or one
lane per node and component (bit-identical results).  Small grids want small
tiles and two lanes (more wavefronts to cover the 256 compute units and
shorter per-lane work); large grids want taller tiles and one lane (a
smaller density halo per node, fewer instructions per byte).  The tuner
times a few steps of the caller's own problem for each candidate on the
device and keeps the fastest, cached per (storage, BC, grid-size bucket) for
the life of the process and in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time

from .sim import Batch, Simulation

# (tile rows, lanes per node)
CANDIDATES = ((4, 1), (8, 1), (16, 1), (32, 1), (4, 2), (8, 2), (16, 2))
_CACHE_PATH = os.path.join(os.path.expanduser("~"), ".cache", "mclbm", "autotune-v3.json")
_cache = None


def _load():
    global _cache
    if _cache is None:
        try:
            with open(_CACHE_PATH) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def _save():
    try:
        os.makedirs(os.path.dirname(_CACHE_PATH), exist_ok=True)
        with open(_CACHE_PATH, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)
    except OSError:
        pass


def bucket(n: int) -> int:
    """Grid sizes are bucketed by powers of two."""
    return 1 << max(0, int(math.ceil(math.log2(max(1, n)))))


def key_of(nx, ny, bc, storage):
    return "%s-bc%d-%dx%d" % (storage, int(bc), bucket(nx), bucket(ny))


def _time(step, sync, steps, reps=3):
    """Best of `reps` timings of `steps` steps, after one untimed run of them
    (which also captures the step graph)."""
    step(steps)
    sync()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        step(steps)
        sync()
        best = min(best, time.perf_counter() - t0)
    return best


def launch_config_for(mask, rhoA0, rhoB0, *, storage="f32", steps=None, stream=None, refresh=False, **params):
    """Fastest {"tile_y", "lanes"} for one simulation of this problem (timed on the device)."""
    import torch

    ny, nx = mask.shape
    key = key_of(nx, ny, params.get("bc", 0), storage)
    cache = _load()
    if key in cache and not refresh:
        return dict(cache[key])
    nodes = nx * ny
    # whole graphs of up to 100 steps, so that host launch cost stays out of
    # the comparison on small grids
    steps = steps or max(20, min(400, int(4e8 / max(nodes, 1))))
    graph = min(100, steps)
    steps = steps // graph * graph
    best, best_t = CANDIDATES[0], float("inf")
    for ty, lanes in CANDIDATES:
        sim = Simulation(mask, rhoA0, rhoB0, stream=stream, storage=storage, tile_y=ty, lanes=lanes,
                         graph_steps=graph, **params)
        t = _time(sim.step, torch.cuda.synchronize, steps)
        sim.close()
        if t < best_t:
            best, best_t = (ty, lanes), t
    cache[key] = dict(tile_y=best[0], lanes=best[1])
    _save()
    return dict(cache[key])


def tile_y_for(mask, rhoA0, rhoB0, **kw):
    """Tile rows of launch_config_for."""
    return launch_config_for(mask, rhoA0, rhoB0, **kw)["tile_y"]


def launch_config_for_batch(items, *, storage="f32", steps=50, stream=None):
    """Fastest {"tile_y", "lanes"} for a batch (one shape for all its instances)."""
    import torch

    # timed without the fused diagnostics (their cadence need not fit these graphs)
    items = [(m, a, b, dict(p, diag_every=0)) for m, a, b, p in items]
    best, best_t = CANDIDATES[0], float("inf")
    for ty, lanes in CANDIDATES:
        b = Batch(items, storage=storage, tile_y=ty, lanes=lanes, stream=stream, graph_steps=steps)
        t = _time(b.step, torch.cuda.synchronize, steps)
        b.close()
        if t < best_t:
            best, best_t = (ty, lanes), t
    return dict(tile_y=best[0], lanes=best[1])
