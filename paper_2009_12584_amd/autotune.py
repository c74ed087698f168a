"""Launch-shape autotuner for the step kernels.

A tile is 64 nodes wide (one wavefront row) and TY rows tall, TY in
{4, 8, 16, 32}; the two-component step runs with one lane per node or one
lane per node and component (bit-identical results).  The 64 x 8 tile with
one lane per node (one thread per node) is the default with FP32 storage: on
MI355X it is the fastest or within 2% of the fastest on every FP32 workload
measured, from the latency-bound 512 x 256 plane to the 5600 x 4000 grid;
smaller tiles and two lanes win only where few tiles cover the 256 compute
units.  With FP16 storage the two-component step defaults to the 64 x 16
tile (four nodes per thread): a node moves half the bytes, and four per thread keep enough of them
in flight (2.6% to 7% faster than 64 x 8 on the 5600 x 4000 grids and the
64-instance batch).  The library applies the same defaults.  The tuner times
a few steps of the caller's own problem for each candidate on the device and
keeps the default unless another shape is at least 2% faster (shapes within
timing noise of each other would otherwise flip from run to run), cached per
(storage, BC, grid-size bucket) for the life of the process and in a JSON
file.
"""
from __future__ import annotations

import json
import math
import os
import time

from .sim import Batch, Simulation

# (tile rows, lanes per node)
CANDIDATES = ((8, 1), (4, 1), (16, 1), (32, 1), (4, 2), (8, 2), (16, 2))
MARGIN = 0.02  # another shape must be this much faster than the default


def default_shape(storage="f32", model=0):
    """The library's own choice when tile_y and lanes are left at 0."""
    return (16, 1) if storage == "f16" and model == 0 else (8, 1)


_CACHE_PATH = os.path.join(os.path.expanduser("~"), ".cache", "mclbm", "autotune-v5.json")
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


def pick(times, storage="f32", model=0):
    """The default shape of the storage and model unless another is at least
    MARGIN faster; then the fastest."""
    default = default_shape(storage, model)
    fastest = min(times, key=times.get)
    if default in times and times[fastest] > (1.0 - MARGIN) * times[default]:
        return default
    return fastest


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
    times = {}
    for ty, lanes in CANDIDATES:
        sim = Simulation(mask, rhoA0, rhoB0, stream=stream, storage=storage, tile_y=ty, lanes=lanes,
                         graph_steps=graph, **params)
        times[(ty, lanes)] = _time(sim.step, torch.cuda.synchronize, steps)
        sim.close()
    best = pick(times, storage, params.get("model", 0))
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
    times = {}
    for ty, lanes in CANDIDATES:
        b = Batch(items, storage=storage, tile_y=ty, lanes=lanes, stream=stream, graph_steps=steps)
        times[(ty, lanes)] = _time(b.step, torch.cuda.synchronize, steps)
        b.close()
    best = pick(times, storage, items[0][3].get("model", 0) if items else 0)
    return dict(tile_y=best[0], lanes=best[1])
