"""Tile-shape autotuner for the step kernels.

A tile is 64 nodes wide (one wavefront per row) and TY rows tall, TY in
{4, 8, 16}.  Small grids want small tiles (more workgroups to cover the 256
compute units); large grids want taller tiles (a smaller density halo per
node).  The tuner times a few steps of the caller's own problem for each
candidate on the device and keeps the fastest, cached per (storage, BC,
grid-size bucket) for the life of the process and in a JSON file.
"""
from __future__ import annotations

import json
import math
import os
import time

from .sim import Batch, Simulation

CANDIDATES = (4, 8, 16, 32)
_CACHE_PATH = os.path.join(os.path.expanduser("~"), ".cache", "mclbm", "autotune.json")
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


def _time(step, sync, steps):
    step(4)
    sync()
    t0 = time.perf_counter()
    step(steps)
    sync()
    return time.perf_counter() - t0


def tile_y_for(mask, rhoA0, rhoB0, *, storage="f32", steps=None, stream=None, refresh=False, **params):
    """Best tile height for one simulation of this problem (timed on the device)."""
    import torch

    ny, nx = mask.shape
    key = key_of(nx, ny, params.get("bc", 0), storage)
    cache = _load()
    if key in cache and not refresh:
        return int(cache[key])
    nodes = nx * ny
    steps = steps or max(20, min(400, int(4e8 / max(nodes, 1))))
    best, best_t = CANDIDATES[0], float("inf")
    for ty in CANDIDATES:
        sim = Simulation(mask, rhoA0, rhoB0, stream=stream, storage=storage, tile_y=ty, **params)
        t = _time(sim.step, torch.cuda.synchronize, steps)
        sim.close()
        if t < best_t:
            best, best_t = ty, t
    cache[key] = best
    _save()
    return best


def tile_y_for_batch(items, *, storage="f32", steps=50, stream=None):
    """Best tile height for a batch (one height for all its instances)."""
    import torch

    best, best_t = CANDIDATES[0], float("inf")
    for ty in CANDIDATES:
        b = Batch(items, storage=storage, tile_y=ty, stream=stream)
        t = _time(b.step, torch.cuda.synchronize, steps)
        b.close()
        if t < best_t:
            best, best_t = ty, t
    return best
