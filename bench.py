"""Benchmark of the two-component wetting LBM step on one MI355X.

Headline workload: 512 x 256 lattice, 30-degree stair wall, drop R = 40 at
rest, improved virtual solid density scheme (D2Q25 average), FP32 deviation
storage -- the set-up of the paper's Section 3 at the size the headline
metric is quoted on.  One bench "step" is one lattice time step of the whole
hot path: pull streaming with bounce-back, densities, virtual solid
densities, forces, velocity, collision, store, and the fused FP64
diagnostics at their cadence (every 100 steps, with the mass-drift check).

Also reported (same JSON line):
  copy_probe              plain streaming copy: the practical HBM ceiling
  roofline_out_of_cache   the same kernel on the paper's largest grid,
                          5600 x 4000 (3.2 GB per step, out of every cache)
  batched                 64 uneven instances, one launch per step (HIP graph)
                          against the plain per-instance loop, FP32 and FP16
  served                  Poisson request stream through the resident pool
                          with continuous batching: p50/p99 latency, MLUPS,
                          against running the same requests one by one
  single_component        the single-component multiphase model on the same
                          5600 x 4000 grid (9 populations per node)
  cpu_baseline            the FP64 oracle on the host cores, bounded sample

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 18 populations read + written per fluid node; with FP16 storage the two
# rest populations stay FP32 (16 FP16 + 2 FP32 values each way)
BYTES_PER_FLUID = {"f32": 144, "f16": 80}
BYTES_PER_FLUID_SC1 = {"f32": 72, "f16": 40}  # 9 populations read + written, single-component model
BYTES_PER_NODE_FLAGS = 2                     # one 16-bit node word per node
KERNEL_SOURCES = ["lbm_device.hpp", "lbm_pair.hpp", "lbm_sc1.hpp", "lbm_common.hpp", "lbm_single.hip",
                  "lbm_batch.hip"]


def alg_bytes(fluid, nodes, storage="f32"):
    return BYTES_PER_FLUID[storage] * fluid + BYTES_PER_NODE_FLAGS * nodes


def kernel_source_hash():
    h = hashlib.sha256()
    for n in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_12584_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, profile):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on the copy
    probe) from a committed rocprofv3 summary in profiles/, if it was taken on
    the current kernel sources; else None."""
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    m = re.search(r"kernel source hash: `([0-9a-f]+)`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    section = text.split("## HBM traffic", 1)
    if len(section) < 2:
        return None
    m = re.search(r"^\| %s \| ([0-9.]+) \| ([0-9.]+) \| ([0-9.]+) \|" % re.escape(name), section[1], re.M)
    return round(float(m.group(3)) * 1e6) if m else None


class Timer:
    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.e0.record(self.stream)
        return self

    def __exit__(self, *exc):
        self.e1.record(self.stream)
        self.torch.cuda.synchronize()
        self.ms = self.e0.elapsed_time(self.e1)


def copy_probe(torch, nbytes=1 << 31, reps=5):
    import ctypes

    from paper_2009_12584_amd import capi

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    st = torch.cuda.current_stream()
    go = lambda: capi.check(capi.lib().lbm_copy_probe(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                                      nbytes, ctypes.c_void_p(st.cuda_stream)))
    go()
    with Timer(torch, st) as t:
        for _ in range(reps):
            go()
    ms = t.ms / reps
    del a, b
    return {"bytes_read_plus_written": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / ms / 1e6, 1),
            "frac_of_peak": round(2 * nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)}


def run_single(M, torch, case, mask, steps, warmup, *, storage="f32", tile_y=0, lanes=0, graph_steps=100,
               diag_every=100):
    stream = torch.cuda.Stream()
    sim = M.Simulation(mask, case.rhoA0, case.rhoB0, stream=stream, storage=storage, graph_steps=graph_steps,
                       diag_every=diag_every, drift_tol=1e-3, tile_y=tile_y, lanes=lanes, **case.params())
    sim.step(warmup)
    if graph_steps:
        steps = max(graph_steps, steps // graph_steps * graph_steps)  # whole graph replays only
    with Timer(torch, stream) as t:
        sim.step(steps)
    d = sim.diag()
    sim.close()
    return dict(steps=steps, ms=t.ms, diag=d)


def batched_rows(M, torch, W, steps=1000):
    from paper_2009_12584_amd.autotune import launch_config_for_batch

    cases = W.config4_instances(64)
    masks = [M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]
    items = [(m, c.rhoA0, c.rhoB0, c.params()) for m, c in zip(masks, cases)]
    fluid = sum(int((m == 0).sum()) for m in masks)
    out = {"workload": "64 seeded instances, W in 128..768, H in 64..384, beta in [0,45] deg, BC uniform among "
                       "the three, drop R=H/5, %d steps" % steps, "fluid_nodes": fluid}
    stream = torch.cuda.Stream()
    # plain per-instance loop: each simulation alone, one after the other (each with its own graph)
    sims = [M.Simulation(m, c.rhoA0, c.rhoB0, stream=stream, graph_steps=100, **c.params())
            for m, c in zip(masks, cases)]
    for s in sims:
        s.step(100)
    with Timer(torch, stream) as t:
        for s in sims:
            s.step(steps)
    plain_ms = t.ms
    ref = [sims[k].fields() for k in (0, 1, 2)]
    for s in sims:
        s.close()
    out["plain_loop_fluid_mlups"] = round(fluid * steps / (plain_ms * 1e-3) / 1e6, 1)
    for storage in ("f32", "f16"):
        cfg = launch_config_for_batch(items, storage=storage, stream=stream)
        ty = cfg["tile_y"]
        b = M.Batch(items, storage=storage, graph_steps=100, tile_y=ty, lanes=cfg["lanes"], stream=stream)
        b.step(100)
        with Timer(torch, stream) as t:
            b.step(steps)
        mlups = fluid * steps / (t.ms * 1e-3) / 1e6
        row = {"fluid_mlups": round(mlups, 1), "ms_per_step": t.ms / steps, "tile_y": ty, "lanes": cfg["lanes"],
               "speedup_vs_plain_loop": round(mlups / out["plain_loop_fluid_mlups"], 2),
               "hbm_gbs_algorithmic": round(alg_bytes(fluid, 0, storage) / (t.ms / steps * 1e-3) / 1e9, 1),
               "hbm_frac": round(alg_bytes(fluid, 0, storage) / (t.ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        if storage == "f16":
            # FP16 error against the FP32 run of the same instances (same step count)
            errs = []
            for k in (0, 1, 2):
                g = b.fields(k)
                fl = masks[k] == 0
                errs.append(float(max((abs(g[0] - ref[k][0])[fl] / ref[k][0][fl]).max(),
                                      (abs(g[1] - ref[k][1])[fl] / ref[k][1][fl]).max())))
            row["max_rel_rho_diff_vs_fp32"] = max(errs)
        out[storage] = row
        b.close()
    return out


def served_rows(M, torch, W, n_req=40, chunk=200):
    from paper_2009_12584_amd.serve import Request, serve, summarize

    reqs = []
    for t, c in W.config5_requests(n=n_req):
        m = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
        reqs.append(Request(t, m, c.rhoA0, c.rhoB0, c.steps, c.params(), tag=c.name))
    stream = torch.cuda.Stream()
    done, makespan = serve(reqs, hbm_budget=48 << 30, max_slots=64, chunk=chunk, stream=stream)
    s = summarize(done, makespan)
    # the same requests run one at a time; their completion latencies under a
    # first-come first-served queue follow from the arrival times and the
    # measured service time of each request
    lu = 0
    service = []
    for r in reqs:
        with Timer(torch, stream) as t:
            sim = M.Simulation(r.mask, r.rhoA0, r.rhoB0, stream=stream, graph_steps=100, **r.params)
            sim.step(r.steps)
            sim.fields()
            sim.close()
        service.append(t.ms * 1e-3)
        lu += int((r.mask == 0).sum()) * r.steps
    plain = lu / sum(service) / 1e6
    by_arrival = sorted(zip(reqs, service), key=lambda rs: rs[0].arrival)

    def fifo_latencies(scale):
        free, lat = 0.0, []
        for r, sv in by_arrival:
            free = max(free, r.arrival * scale) + sv
            lat.append(free - r.arrival * scale)
        return sorted(lat)

    lat = fifo_latencies(1.0)
    pct = lambda q, lat=lat: lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
    s.update({"workload": "%d requests, Poisson 200/s, W in 64..2048, H in 64..1024, 2k-20k steps, mixed BCs "
                          "and angles, FP32, chunk %d steps" % (n_req, chunk),
              "hbm_gbs_algorithmic": round(s["fluid_mlups"] * BYTES_PER_FLUID["f32"] / 1e3, 1),
              "hbm_frac": round(s["fluid_mlups"] * BYTES_PER_FLUID["f32"] / 1e3 / HBM_PEAK_GBS, 4),
              "accuracy": "each result bit-identical alone and in the mix, FP32 (GPU tests)",
              "plain_loop_fluid_mlups": round(plain, 1), "speedup_vs_plain_loop": round(s["fluid_mlups"] / plain, 2),
              "plain_loop_fifo_p50_latency_s": round(pct(0.5), 4), "plain_loop_fifo_p99_latency_s": round(pct(0.99), 4)})
    for k in ("makespan_s", "p50_latency_s", "p99_latency_s", "mean_latency_s", "fluid_mlups"):
        s[k] = round(s[k], 4)
    # the same trace with 16 slots admitted shortest-job-first: shorter median
    # latency for a little less throughput
    done2, mk2 = serve(reqs, hbm_budget=48 << 30, max_slots=16, chunk=chunk, stream=stream, policy="sjf")
    s2 = summarize(done2, mk2)
    s["sjf_16_slots"] = {k: round(v, 4) for k, v in s2.items()}
    # the same trace with its arrival times stretched so that requests arrive
    # at 80% of the rate the pool sustained above (still a Poisson process):
    # completion latency without a standing backlog; one by one, the same
    # arrivals exceed that server's capacity
    rate = 0.8 * n_req / s["makespan_s"]
    scale = 200.0 / rate  # the trace is Poisson at 200 requests per second
    done3, mk3 = serve(reqs, hbm_budget=48 << 30, max_slots=64, chunk=chunk, stream=stream, time_scale=scale)
    s3 = {k: round(v, 4) for k, v in summarize(done3, mk3).items()}
    lat3 = fifo_latencies(scale)
    p3 = lambda q: lat3[min(len(lat3) - 1, int(round(q * (len(lat3) - 1))))]
    s3.update({"arrival_rate_per_s": round(rate, 3), "plain_loop_fifo_p50_latency_s": round(p3(0.5), 4),
               "plain_loop_fifo_p99_latency_s": round(p3(0.99), 4)})
    s["at_80pct_of_capacity"] = s3
    return s


def headline_row(M, torch, case, mask, fluid, nodes, args, probe, launch_config_for):
    cfg = launch_config_for(mask, case.rhoA0, case.rhoB0, **case.params())
    ty, lanes = cfg["tile_y"], cfg["lanes"]
    gs = 100 if args.graph_steps is None else args.graph_steps
    r = run_single(M, torch, case, mask, args.steps, args.warmup, tile_y=ty, lanes=lanes, graph_steps=gs)
    K = r["steps"]
    ms_per_step = r["ms"] / K
    mlups = fluid * K / (r["ms"] * 1e-3) / 1e6
    kname = "%s<float, %d, 2, 0, false>" % ("k_step_ls" if lanes == 2 else "k_step", ty)
    achieved = alg_bytes(fluid, nodes) / (ms_per_step * 1e-3) / 1e9
    d = r["diag"]
    return {
        "metric": "fluid MLUPS, two-component D2Q9 wetting LBM step",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x256 D2Q9 two-component, 30-degree stair wall, drop R=40, improved virtual "
                               "solid density (D2Q25), tau=1, G=0.9, rho 1.0/0.03, FP32 deviations",
                   "nx": case.nx, "ny": case.ny, "fluid_nodes": fluid, "total_nodes": nodes,
                   "total_mlups": round(nodes * K / (r["ms"] * 1e-3) / 1e6, 1), "tile_y": ty, "lanes": lanes,
                   "graph_steps": gs, "diag_every": 100,
                   "mass_drift": max(abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k] for k in range(2))},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kname, "k_step_improved_plane30_512x256.md"), "kernel": kname,
                     "profile": "profiles/k_step_improved_plane30_512x256.md",
                     "bytes_per_launch": alg_bytes(fluid, nodes),
                     "note": "algorithmic bytes = 144 B per fluid node + 2 B node word per node; the 18.9 MB working set "
                             "stays in L2/Infinity Cache, see roofline_out_of_cache for HBM"},
        "copy_probe": probe,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--large-steps", type=int, default=200)
    ap.add_argument("--rows", default="headline,large,sc1,batched,served,cpu",
                    help="comma list of rows to run (profiling runs select one)")
    ap.add_argument("--served-requests", type=int, default=40)
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps per captured HIP graph in the single-simulation rows (0 = plain launches, "
                         "which per-dispatch counter collection needs); default 100 (headline), 20 (large grids)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the slab decomposition is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_2009_12584_amd as M
    from paper_2009_12584_amd.autotune import launch_config_for

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    rows = set(args.rows.split(","))
    probe = copy_probe(torch)
    out = {}

    case = W.config2()
    mask = M.mask_plane(case.nx, case.ny, case.geometry[1], case.geometry[2])
    fluid = int((mask == 0).sum())
    nodes = case.nx * case.ny
    if "headline" in rows:
        out.update(headline_row(M, torch, case, mask, fluid, nodes, args, probe, launch_config_for))
    else:
        out.update({"metric": "fluid MLUPS, two-component D2Q9 wetting LBM step", "value": None, "unit": "MLUPS",
                    "n_gpus": 1, "steps": 0, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                    "config": {"workload": "headline row skipped (--rows)"}, "copy_probe": probe})

    if "large" in rows:
        big = W.roofline_case()
        bmask = big.mask_user
        bfl = int((bmask == 0).sum())
        lrows = {}
        for storage in ("f32", "f16"):
            bty = 8  # 64 x 8 and 64 x 16 tiles are within 1% here; fixed so profiles name the same kernel
            rb = run_single(M, torch, big, bmask, args.large_steps, 10, storage=storage, tile_y=bty,
                            graph_steps=20 if args.graph_steps is None else args.graph_steps, diag_every=20)
            bms = rb["ms"] / rb["steps"]
            bach = alg_bytes(bfl, big.nx * big.ny, storage) / (bms * 1e-3) / 1e9
            kn = "k_step<%s, %d, 0, 0, false>" % ("float" if storage == "f32" else "__half", bty)
            lrows[storage] = {"achieved": round(bach, 1), "frac": round(bach / HBM_PEAK_GBS, 4),
                              "frac_of_copy_probe": round(bach / probe["gbs"], 4), "ms_per_step": round(bms, 4),
                              "fluid_mlups": round(bfl * rb["steps"] / (rb["ms"] * 1e-3) / 1e6, 1), "tile_y": bty,
                              "kernel": kn, "bytes_per_launch": alg_bytes(bfl, big.nx * big.ny, storage),
                              "traffic": measured_traffic(kn, "k_step_mc_periodic_5600x4000.md"),
                              "profile": "profiles/k_step_mc_periodic_5600x4000.md"}
        out["roofline_out_of_cache"] = dict(
            workload="5600x4000 fully periodic G=3 mixture (Martys-Chen path), 3.2 GB ping-pong in FP32",
            bound="hbm", peak=HBM_PEAK_GBS, unit="GB/s", **lrows["f32"], f16=lrows["f16"])

    if "sc1" in rows:
        sc = W.sc1_roofline_case()
        sfl = sc.nx * sc.ny
        srows = {}
        for storage in ("f32", "f16"):
            rs = run_single(M, torch, sc, sc.mask_user, args.large_steps, 10, storage=storage, tile_y=8,
                            graph_steps=20 if args.graph_steps is None else args.graph_steps, diag_every=20)
            sms = rs["ms"] / rs["steps"]
            sb = BYTES_PER_FLUID_SC1[storage] * sfl + BYTES_PER_NODE_FLAGS * sfl
            kn = "k_step_sc1<%s, 8, 0, 0, false>" % ("float" if storage == "f32" else "__half")
            srows[storage] = {"achieved": round(sb / (sms * 1e-3) / 1e9, 1),
                              "frac": round(sb / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "ms_per_step": round(sms, 4),
                              "fluid_mlups": round(sfl * rs["steps"] / (rs["ms"] * 1e-3) / 1e6, 1), "kernel": kn,
                              "bytes_per_launch": sb, "traffic": measured_traffic(kn, "k_step_sc1_periodic_5600x4000.md"),
                              "profile": "profiles/k_step_sc1_periodic_5600x4000.md"}
        out["single_component"] = dict(
            workload="5600x4000 fully periodic single-component Shan-Chen at G=-5 (liquid-vapour separation), "
                     "Martys-Chen path", bound="hbm", peak=HBM_PEAK_GBS, unit="GB/s", **srows["f32"], f16=srows["f16"])

    if "batched" in rows:
        out["batched"] = batched_rows(M, torch, W)

    if "served" in rows:
        out["served"] = served_rows(M, torch, W, n_req=args.served_requests)

    if "cpu" in rows:
        import oracle

        oracle.build()
        o = oracle.Oracle(mask, case.rhoA0, case.rhoB0, **case.params())
        o.step(5)
        n = 6000
        t0 = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(fluid * n / dt / 1e6, 2), "unit": "MLUPS", "cores": oracle.threads(),
                               "kind": "oracle",
                               "sample": "same 512x256 workload, %d steps of the FP64 C oracle (%.1f s wall)" % (n, dt)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
