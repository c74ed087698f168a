"""Served form: a request loop over the resident-slot pool (continuous batching).

Requests arrive on a wall clock; each carries its wall mask, initial densities,
parameters and step count.  The loop admits requests first-come first-served
whenever the pool has a free slot and HBM budget (lbm_pool_admit), advances
every active slot together in chunks of time steps (lbm_pool_advance: one
batched launch per step; new slots join at the next chunk while older ones
keep running), and retires finished slots (lbm_pool_poll / fields / release)
without stopping the others.  With diag_every > 0 the pool's fused
diagnostics flag a solve that breaks (non-finite or negative density, mass
drift); it is retired at once, marked failed, and the others go on.
Completion latency = retirement time - arrival time.  All stepping happens in
the HIP library; this loop only schedules.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .sim import Pool


@dataclass
class Request:
    arrival: float          # seconds after the start of the trace
    mask: np.ndarray
    rhoA0: np.ndarray
    rhoB0: np.ndarray
    steps: int
    params: dict
    tag: object = None
    fluid: int = 0


@dataclass
class Done:
    tag: object
    arrival: float
    admitted: float
    finished: float
    steps: int
    fluid: int
    fields: tuple | None = field(default=None, repr=False)
    failed: bool = False

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def serve(requests, *, hbm_budget, max_slots, storage="f32", chunk=200, depth=2, keep_fields=False, stream=None,
          time_scale=1.0, idle_sleep=0.0002, policy="fifo", pool_factory=None, clock=None, sleep=None,
          diag_every=0, keep_tags=None):
    """Run the trace; returns (list of Done, makespan seconds).

    At most `depth` chunks are in flight on the device, so a new solve waits
    at most that many chunks before it joins the running batch.  time_scale
    stretches the arrival times (1.0 = as given).  policy picks the next
    waiting request to admit: "fifo" (arrival order) or "sjf" (the smallest
    amount of work, fluid nodes x steps, first); with fewer slots than
    waiting requests, "sjf" finishes short solves early instead of sharing
    the device among everything that has arrived.  pool_factory, clock and
    sleep replace the device pool (Pool's constructor and methods), the wall
    clock (time.perf_counter) and time.sleep, so that the scheduling logic
    can run against a simulated device and clock.  Fields are read back for
    every request with keep_fields, else only for the tags in keep_tags."""
    if policy not in ("fifo", "sjf"):
        raise ValueError("policy must be 'fifo' or 'sjf'")
    now_fn = clock or time.perf_counter
    sleep_fn = sleep or time.sleep
    reqs = sorted(requests, key=lambda r: r.arrival)
    for r in reqs:
        if not r.fluid:
            r.fluid = int((np.asarray(r.mask) == 0).sum())
    pool = (pool_factory or Pool)(hbm_budget, max_slots, storage=storage, diag_every=diag_every, stream=stream)
    queue = []
    live = {}
    done = []
    nxt = 0
    t0 = now_fn()
    try:
        while nxt < len(reqs) or queue or live:
            now = now_fn() - t0
            while nxt < len(reqs) and reqs[nxt].arrival * time_scale <= now:
                queue.append(reqs[nxt])
                nxt += 1
            if policy == "sjf":
                queue.sort(key=lambda q: q.fluid * q.steps)
            while queue:  # admission in policy order while a slot and the budget allow
                r = queue[0]
                slot = pool.admit(r.mask, r.rhoA0, r.rhoB0, r.steps, **r.params)
                if slot is None:
                    break
                live[slot] = (r, now_fn() - t0)
                queue.pop(0)
            if queue and not live:
                # an empty pool that cannot take the next request never will
                raise ValueError("request %r does not fit an empty pool (budget %d B, %d slots)"
                                 % (queue[0].tag, hbm_budget, max_slots))
            if live:
                launched, completed = pool.progress()
                if launched - completed < depth * chunk:
                    pool.advance(chunk)
            finished = pool.poll() if live else []
            for slot in finished:
                r, ta = live.pop(slot)
                failed = pool.status(slot) != 0
                keep = keep_fields or (keep_tags is not None and r.tag in keep_tags)
                f = pool.fields(slot, raise_on_flags=False) if keep else None
                pool.release(slot)
                done.append(Done(r.tag, r.arrival * time_scale, ta, now_fn() - t0, r.steps, r.fluid, f, failed))
            if not finished and not queue and nxt < len(reqs) and not live:
                # nothing to do until the next arrival
                sleep_fn(max(0.0, min(0.01, reqs[nxt].arrival * time_scale - (now_fn() - t0))))
            elif not finished and live:
                sleep_fn(idle_sleep)
        makespan = now_fn() - t0
    finally:
        pool.close()
    return done, makespan


def percentile(values, q):
    """The percentile rule every latency summary here uses: linear
    interpolation between order statistics (numpy's default)."""
    return float(np.percentile(np.asarray(values, dtype=float), q))


def summarize(done, makespan):
    lat = [d.latency for d in done]
    lu = float(sum(d.fluid * d.steps for d in done if not d.failed))
    return dict(requests=len(done), failed=sum(1 for d in done if d.failed), makespan_s=makespan,
                p50_latency_s=percentile(lat, 50), p99_latency_s=percentile(lat, 99),
                mean_latency_s=float(np.mean(lat)), fluid_mlups=lu / makespan / 1e6)
