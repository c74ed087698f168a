"""Benchmark of the two-component wetting LBM step on one MI355X.

Headline workload: configuration 3, the largest single-instance one: a
1024 x 1024 lattice with a solid disk of radius 300 at its centre and two
drops of radius 60 touching on its top (the coalescence set-up of the
paper's Section 4), improved virtual solid density scheme (Eq. 7, D2Q25
average, chi^A = 2s, chi^B = 2 - 2s with the seed-0 solid density s), FP32
deviation storage.  One bench "step" is one lattice time step of the whole
hot path: pull streaming with bounce-back, densities, virtual solid
densities, forces, velocity, collision, store, and the fused FP64
diagnostics (mass, momentum, drift check) at their cadence.  --steps K are
timed exactly, after --warmup W steps and the few untimed steps that bring
the time to a multiple of the graph length (graphs replay only from there);
the line reports how many of the K steps ran in graph replays.  The run then
continues, untimed, to the configuration's 50,000 steps, where its fields are
compared with the FP64 oracle's (tests/golden/longrun_c3.npz, written by the
oracle alone).

Roofline: achieved = algorithmic bytes per launch / the average time per
launch over the timed region (HIP events on the simulation's stream); the
algorithmic bytes per fluid lattice update are those of the survey's
measurement table, 145 B in FP32 (18 populations read and written, 4 B each,
plus the 1-byte mask) and 73 B in FP16.  traffic = FETCH_SIZE + WRITE_SIZE
per launch from the committed counter summary in profiles/, when it was taken
on the current kernel sources (else null).

Also reported (same JSON line):
  copy_probe       plain streaming copy: the practical HBM ceiling
  rows_5600x4000   the paper's largest grid (Section 4), out of every cache:
                   the periodic G = 3 mixture (FP32, FP16), a drop on a
                   30-degree stair plane in each wetting rule (FP32) and in
                   the improved scheme in FP16, the single-component model;
                   each with its error against the oracle on three 240 x 240
                   windows after 10 steps of the same run
  config2          the 512 x 256 plane of configuration 2 (latency-bound)
  batched          configuration 4: 64 uneven instances, one launch per step,
                   against the plain per-instance loop, FP32 and FP16, with
                   the error of four instances against the oracle
  served           configuration 5: the 400-request Poisson trace through the
                   resident pool (continuous batching), p50/p99 latency and
                   MLUPS, under the trace's overload and at 80% of the pool's
                   capacity, against the same requests served one by one
  cpu_baseline     the FP64 oracle on the host cores (all threads and one)

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (2-comp D2Q9) + % HBM peak; batched/served p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid lattice update (survey measurement table)
ALG_BYTES = {"f32": 145, "f16": 73}
ALG_BYTES_SC1 = {"f32": 73, "f16": 37}  # single-component: 9 populations each way + mask
# what this design moves: FP16 storage keeps both rest populations in FP32;
# one 2-byte node word is read per node
DESIGN_BYTES_FLUID = {"f32": 144, "f16": 80}
DESIGN_BYTES_FLUID_SC1 = {"f32": 72, "f16": 40}
DESIGN_BYTES_NODE = 2
KERNEL_SOURCES = ["lbm_tiling.hpp", "lbm_plan.hpp", "lbm_device.hpp", "lbm_pair.hpp", "lbm_sc1.hpp",
                  "lbm_common.hpp", "lbm_step_kernels.hpp", "lbm_batch_kernels.hpp", "lbm_single.hip",
                  "lbm_step_f32.hip", "lbm_step_f16.hip", "lbm_batch.hip", "lbm_batch_f32.hip", "lbm_batch_f16.hip"]
RHO_TOL, U_TOL = 1e-5, 1e-6            # FP32 bar against the FP64 oracle
RHO_TOL_F16, U_TOL_F16 = 5e-3, 1e-3   # FP16 bar (derived from the storage rounding)


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


def roofline(kernel, profile, fluid, nodes, storage, ms_per_launch, sc1=False):
    alg = (ALG_BYTES_SC1 if sc1 else ALG_BYTES)[storage] * fluid
    des = (DESIGN_BYTES_FLUID_SC1 if sc1 else DESIGN_BYTES_FLUID)[storage] * fluid + DESIGN_BYTES_NODE * nodes
    gbs = alg / (ms_per_launch * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, profile), "kernel": kernel,
            "profile": "profiles/" + profile, "alg_bytes_per_launch": alg, "design_bytes_per_launch": des,
            "design_frac": round(des / (ms_per_launch * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


# the library's store policy: streaming (non-temporal) population stores only
# when both population buffers together exceed 192 MiB; smaller grids keep
# their populations in the 256 MB Infinity Cache between steps
NT_STORE_BYTES = 192 << 20


def streaming_stores(nx, ny, storage, comps=2):
    pitch = (nx + 63) // 64 * 64
    per_node = 9 * 4 if storage == "f32" else 9 * 2 + 4
    return 2 * comps * ny * pitch * per_node > NT_STORE_BYTES


def kernel_name(storage, ty, lanes, bc, nx, ny, sc1=False):
    s = "float" if storage == "f32" else "__half"
    nt = "true" if streaming_stores(nx, ny, storage, 1 if sc1 else 2) else "false"
    if sc1:
        return "k_step_sc1<%s, %d, %d, 0, false, %s>" % (s, ty, bc, nt)
    return "%s<%s, %d, %d, 0, false, %s>" % ("k_step_ls" if lanes == 2 else "k_step", s, ty, bc, nt)


class Timer:
    """HIP events on the stream the kernels are launched on."""

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


def errors(mask, got, ref):
    """Max relative rho error over both components and max absolute u error, on fluid nodes."""
    import numpy as np

    fl = mask == 0
    er = max(float(np.max(np.abs(got[0] - ref[0])[fl] / ref[0][fl])), float(np.max(np.abs(got[1] - ref[1])[fl] / ref[1][fl])))
    eu = max(float(np.max(np.abs(got[2] - ref[2])[fl])), float(np.max(np.abs(got[3] - ref[3])[fl])))
    return er, eu


def err_entry(er, eu, storage, bar=None, **extra):
    rt, ut = bar if bar else ((RHO_TOL, U_TOL) if storage == "f32" else (RHO_TOL_F16, U_TOL_F16))
    return dict(max_rel_rho=float("%.3e" % er), max_abs_u=float("%.3e" % eu), bar=[float("%.3e" % rt),
                float("%.3e" % ut)], within_bar=bool(er <= rt and eu <= ut), **extra)


def f16_model_bars(W, cases, masks, picks, at_step):
    """Per picked instance, twice the error FP16 storage alone gives at
    at_step (the FP64 oracle with the storage rounding applied,
    tests/golden/f16_model_c4.npz, written by the oracle alone); None when
    the file does not cover the instances or the step."""
    import numpy as np

    try:
        gold = np.load(os.path.join(ROOT, "tests", "golden", "f16_model_c4.npz"), allow_pickle=False)
    except OSError:
        return None
    steps = [int(x) for x in gold["steps"]]
    inst = [int(x) for x in gold["instances"]]
    if at_step not in steps or any(k not in inst for k in picks):
        return None
    col = steps.index(at_step)
    out = {}
    for k in picks:
        if str(gold["input_sha_%d" % k]) != W.input_hash(cases[k], masks[k]):
            return None
        a = inst.index(k)
        out[k] = (2 * float(gold["err_rho"][a, col]), 2 * float(gold["err_u"][a, col]))
    return out


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


def graph_len(args, steps):
    """Steps per captured graph: 0 (plain launches) when --graph-steps 0, else
    --graph-steps or min(100, steps), rounded up to even."""
    if args.graph_steps == 0:
        return 0
    g = args.graph_steps if args.graph_steps else min(100, max(2, steps))
    return (g + 1) // 2 * 2


# ----------------------------------------------------------------- headline

def headline(M, torch, W, args, probe):
    import numpy as np
    from paper_2009_12584_amd.autotune import launch_config_for

    c = W.config3(0)
    g = c.geometry
    mask = M.mask_disk(c.nx, c.ny, g[1], g[2], g[3])
    fluid, nodes = int((mask == 0).sum()), c.nx * c.ny
    if args.autotune_shapes:
        cfg = launch_config_for(mask, c.rhoA0, c.rhoB0, **c.params())
        ty, lanes = cfg["tile_y"], cfg["lanes"]
    else:
        # the autotuner's pick for this workload on MI355X (64 x 8 tiles, one
        # lane per node: 23.8 us per step against 24.7 for 64 x 4 and 29.6
        # for two lanes), fixed so that the profiled kernel is the timed one
        ty, lanes = 8, 1
    K, Wm = args.steps, args.warmup
    glen = graph_len(args, K)
    diag_every = glen if glen else 100
    stream = torch.cuda.Stream()
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0, stream=stream, graph_steps=glen, diag_every=diag_every,
                       drift_tol=1e-4, tile_y=ty, lanes=lanes, **c.params())
    sim.step(Wm)
    pad = (-sim.t) % glen if glen else 0
    sim.step(pad)
    before = sim.launch_counts()
    with Timer(torch, stream) as t:
        sim.step(K)
    after = sim.launch_counts()
    ms = t.ms / K
    # the rest of the configuration's run, untimed, and the oracle comparison at its final step
    err = None
    if sim.t <= c.steps and not args.no_oracle:
        sim.step(c.steps - sim.t)
        gold = np.load(os.path.join(ROOT, "tests", "golden", "longrun_c3.npz"), allow_pickle=False)
        if str(gold["input_sha"]) == W.input_hash(c, mask):
            idx = gold["idx"]
            got = [f.ravel()[idx] for f in sim.fields()]
            ref = [gold["%s_%d" % (k, c.steps)].astype(np.float64) for k in ("rhoA", "rhoB", "ux", "uy")]
            er, eu = errors(np.zeros(idx.size, np.uint8), got, ref)
            err = err_entry(er, eu, "f32", at_step=c.steps, nodes="%d sampled fluid nodes" % idx.size)
    d = sim.diag()
    sim.close()
    kname = kernel_name("f32", ty, lanes, 2, c.nx, c.ny)
    return {
        "metric": METRIC,
        "value": round(fluid * K / (t.ms * 1e-3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 D2Q9 two-component, solid disk R=300 at the centre, two tanh drops R=60 "
                               "touching on its top, improved virtual solid density (D2Q25), solid density s of "
                               "seed 0 (chi^A=2s, chi^B=2-2s), tau=1, G=0.9, rho 1.0/0.03, FP32 deviations",
                   "nx": c.nx, "ny": c.ny, "fluid_nodes": fluid, "total_nodes": nodes,
                   "total_mlups": round(nodes * K / (t.ms * 1e-3) / 1e6, 1), "tile_y": ty, "lanes": lanes,
                   "graph_steps": glen, "diag_every": diag_every, "alignment_steps": pad,
                   "timed_steps_in_graphs": after["graph_steps"] - before["graph_steps"],
                   "timed_steps_plain": after["plain_steps"] - before["plain_steps"],
                   "mass_drift": max(abs(d["mass"][k] - d["mass0"][k]) / d["mass0"][k] for k in range(2)),
                   "mass_drift_at_step": int(d["step"])},
        "roofline": dict(roofline(kname, "k_step_improved_disk_1024x1024.md", fluid, nodes, "f32", ms),
                         note="151 MB of populations: the step runs out of the 256 MB Infinity Cache; "
                              "rows_5600x4000 give the HBM-bound rows"),
        "error_vs_oracle": err,
        "copy_probe": probe,
    }


# ------------------------------------------------------------ 5600 x 4000 rows

def window_errors(ora, c, mask, fields, windows, size=240, k=10):
    """Error against the oracle after k steps on periodic windows of the
    initial state: a node's state after k steps depends only on the initial
    state within 4 k nodes, so a window's interior beyond that margin is the
    full run's."""
    import numpy as np

    two = c.model == 0
    margin = 4 * k + 2
    worst = (0.0, 0.0)
    for (x0, y0) in windows:
        xs = (np.arange(size) + x0) % c.nx
        ys = (np.arange(size) + y0) % c.ny
        cut = np.ix_(ys, xs)
        prm = c.params()
        prm["periodic"] = 3
        o = ora.Oracle(mask[cut], c.rhoA0[cut], c.rhoB0[cut] if two else None, **prm)
        o.step(k)
        of = o.fields()
        sl = (slice(margin, size - margin),) * 2
        fl = mask[cut][sl] == 0
        got = [f[cut][sl] for f in fields]
        ref = [f[sl] for f in of]
        er = float(np.max(np.abs(got[0] - ref[0])[fl] / ref[0][fl]))
        if two:
            er = max(er, float(np.max(np.abs(got[1] - ref[1])[fl] / ref[1][fl])))
        eu = max(float(np.max(np.abs(got[2] - ref[2])[fl])), float(np.max(np.abs(got[3] - ref[3])[fl])))
        worst = (max(worst[0], er), max(worst[1], eu))
    return worst


def large_row(M, torch, ora, args, c, mask, storage, profile, windows, sc1=False):
    from paper_2009_12584_amd.autotune import default_shape

    fluid, nodes = int((mask == 0).sum()), c.nx * c.ny
    steps = args.large_steps
    glen = graph_len(args, 20)
    stream = torch.cuda.Stream()
    # the library's default tile for the storage: 64 x 8, or 64 x 16 for the
    # two-component step with FP16 storage
    ty = default_shape(storage, 1 if sc1 else 0)[0]
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0 if not sc1 else None, stream=stream, storage=storage, tile_y=ty,
                       lanes=1, graph_steps=glen, diag_every=glen if glen else 20, **c.params())
    sim.step(10)
    er, eu = window_errors(ora, c, mask, sim.fields(), windows) if ora is not None else (float("nan"),) * 2
    sim.step((-sim.t) % glen if glen else 0)
    with Timer(torch, stream) as t:
        sim.step(steps)
    sim.close()
    ms = t.ms / steps
    row = {"ms_per_step": round(ms, 4), "fluid_mlups": round(fluid * steps / (t.ms * 1e-3) / 1e6, 1),
           "fluid_nodes": fluid,
           "tile_y": ty,
           "roofline": roofline(kernel_name(storage, ty, 1, c.bc if c.bc < 3 else 0, c.nx, c.ny, sc1), profile, fluid,
                                nodes, storage, ms, sc1)}
    if ora is not None:
        row["error_vs_oracle"] = err_entry(er, eu, storage, at_step=10, nodes="3 windows of 240 x 240")
    return row


def rows_5600x4000(M, torch, W, args, probe):
    import oracle

    if args.no_oracle:
        oracle = None
    else:
        oracle.build()
    pick = set(args.large_only.split(",")) if args.large_only else None
    out = {"workload": "5600x4000, the paper's largest grid (Section 4): 3.2 GB of FP32 populations per step, "
                       "out of every cache; 64 x 8 tiles (64 x 16 with FP16 storage), one lane per node"}
    mix = W.roofline_case()
    seams = [(5600 - 120, 4000 - 120), (2800, 1900), (5500, 700)]
    for storage in ("f32", "f16"):
        if pick and "mixture_mc_" + storage not in pick:
            continue
        r = large_row(M, torch, oracle, args, mix, mix.mask_user, storage, "k_step_mc_periodic_5600x4000.md", seams)
        r["roofline"]["frac_of_copy_probe"] = round(r["roofline"]["achieved"] / probe["gbs"], 4)
        out["mixture_mc_" + storage] = r
    # the drop touches the plane where the normal through its centre meets it
    wins = [(2800 + 200 - 120, 2000 - 346 - 120), (600, 150), (3000, 3000)]
    for bc, name in ((W.MC, "mc"), (W.LLKC, "llkc"), (W.IMPROVED, "improved")):
        c = W.roofline_plane_case(bc)
        m = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
        for storage in (("f32", "f16") if bc == W.IMPROVED else ("f32",)):
            if pick and "plane30_%s_%s" % (name, storage) not in pick:
                continue
            r = large_row(M, torch, oracle, args, c, m, storage, "k_step_plane30_5600x4000_%s.md" % name, wins)
            r["roofline"]["frac_of_copy_probe"] = round(r["roofline"]["achieved"] / probe["gbs"], 4)
            out["plane30_%s_%s" % (name, storage)] = r
    if not pick or "single_component_f32" in pick:
        sc = W.sc1_roofline_case()
        out["single_component_f32"] = large_row(M, torch, oracle, args, sc, sc.mask_user, "f32",
                                                "k_step_sc1_periodic_5600x4000.md", seams, sc1=True)
    out["plane_workload"] = ("drop R=400 at rest on a 30-degree stair plane (Section 3.1 set-up), G=3, rho 1.0/0.055; "
                             "Martys-Chen G_w=-0.2, LLKC G_w=-0.5, improved chi 1.2/0.8")
    out["mixture_workload"] = "fully periodic seeded 50/50 mixture at G=3 (spinodal start), Martys-Chen path"
    return out


def config2_row(M, torch, W, args):
    from paper_2009_12584_amd.autotune import launch_config_for

    c = W.config2()
    mask = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
    fluid, nodes = int((mask == 0).sum()), c.nx * c.ny
    if args.autotune_shapes:
        cfg = launch_config_for(mask, c.rhoA0, c.rhoB0, **c.params())
        ty, lanes = cfg["tile_y"], cfg["lanes"]
    else:
        # the autotuner's pick (64 x 8, one lane per node: 8.0 us against 8.3
        # for two lanes), fixed so that the profiled kernel is the timed one
        ty, lanes = 8, 1
    glen = graph_len(args, 100)
    stream = torch.cuda.Stream()
    sim = M.Simulation(mask, c.rhoA0, c.rhoB0, stream=stream, graph_steps=glen, diag_every=glen if glen else 100,
                       tile_y=ty, lanes=lanes, **c.params())
    sim.step(200)
    K = args.config2_steps
    with Timer(torch, stream) as t:
        sim.step(K)
    ms = t.ms / K
    # the oracle's fields at the configuration's final step (written by the
    # oracle alone), when the run ends there
    err = None
    if sim.t == c.steps and not args.no_oracle:
        import numpy as np

        gold = np.load(os.path.join(ROOT, "tests", "golden", "longrun_c2.npz"), allow_pickle=False)
        if str(gold["input_sha"]) == W.input_hash(c, mask):
            idx = gold["idx"]
            got = [f.ravel()[idx] for f in sim.fields()]
            ref = [gold["%s_%d" % (k, c.steps)].astype(np.float64) for k in ("rhoA", "rhoB", "ux", "uy")]
            er, eu = errors(np.zeros(idx.size, np.uint8), got, ref)
            err = err_entry(er, eu, "f32", at_step=c.steps, nodes="%d sampled fluid nodes" % idx.size)
    sim.close()
    return {"workload": "512x256, 30-degree stair plane, drop R=40, improved scheme, FP32 (configuration 2); "
                        "18.9 MB of populations: cache-resident and launch-latency-bound",
            "ms_per_step": round(ms, 5), "fluid_mlups": round(fluid * K / (t.ms * 1e-3) / 1e6, 1), "steps": K,
            "tile_y": ty, "lanes": lanes,
            "roofline": roofline(kernel_name("f32", ty, lanes, 2, c.nx, c.ny), "k_step_improved_plane30_512x256.md", fluid,
                                 nodes, "f32", ms),
            "error_vs_oracle": err}


# ----------------------------------------------------------------- batched

def batched_rows(M, torch, W, args):
    import numpy as np
    import oracle
    from paper_2009_12584_amd.autotune import default_shape, launch_config_for_batch

    if not args.no_oracle:
        oracle.build()
    steps = args.batch_steps
    warm = 100
    glen = graph_len(args, 100)
    de = glen if glen else 100
    cases = W.config4_instances(64)
    masks = [M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]
    items = [(m, c.rhoA0, c.rhoB0, dict(c.params(), diag_every=de, drift_tol=1e-4)) for m, c in zip(masks, cases)]
    fluid = sum(int((m == 0).sum()) for m in masks)
    out = {"workload": "64 seeded instances, W in 128..768, H in 64..384, beta in [0,45] deg, BC uniform among "
                       "the three, drop R=H/5, %d steps timed after %d, fused diagnostics every %d" % (steps, warm, de),
           "fluid_nodes": fluid, "graph_steps": glen}
    stream = torch.cuda.Stream()
    # plain per-instance loop: each simulation alone, one after the other
    sims = [M.Simulation(m, c.rhoA0, c.rhoB0, stream=stream, graph_steps=glen, diag_every=de, **c.params())
            for m, c in zip(masks, cases)]
    for s in sims:
        s.step(warm)
    with Timer(torch, stream) as t:
        for s in sims:
            s.step(steps)
    plain_ms = t.ms
    for s in sims:
        s.close()
    out["plain_loop_fluid_mlups"] = round(fluid * steps / (plain_ms * 1e-3) / 1e6, 1)
    picks = () if args.no_oracle else (0, 3, 5)
    refs = {}
    for k in picks:
        o = oracle.Oracle(masks[k], cases[k].rhoA0, cases[k].rhoB0, **cases[k].params())
        o.step(warm + steps)
        refs[k] = o.fields()
    for storage in ("f32", "f16"):
        if args.fixed_shapes or args.graph_steps == 0:
            # the autotuner's default shape: counter runs name one kernel per
            # storage and capture no autotuner graphs
            ty, lanes = default_shape(storage)
        else:
            cfg = launch_config_for_batch(items, storage=storage, stream=stream)
            ty, lanes = cfg["tile_y"], cfg["lanes"]
        b = M.Batch(items, storage=storage, graph_steps=glen, tile_y=ty, lanes=lanes, stream=stream)
        b.step(warm)
        c0 = b.launch_counts()
        with Timer(torch, stream) as t:
            b.step(steps)
        c1 = b.launch_counts()
        ms = t.ms / steps
        worst = (0.0, 0.0)
        # the FP16 bar: twice the FP16 storage format's own error on each
        # instance at this step
        bars = f16_model_bars(W, cases, masks, picks, warm + steps) if storage == "f16" else None
        ok = True
        for k in picks:
            er, eu = errors(masks[k], b.fields(k), refs[k])
            worst = (max(worst[0], er), max(worst[1], eu))
            if bars:
                ok = ok and er <= bars[k][0] and eu <= bars[k][1]
        flags = sum(1 for k in range(64) if b.diag(k, raise_on_flags=False)["flags"])
        b.close()
        mlups = fluid * steps / (t.ms * 1e-3) / 1e6
        kern = ("k_batch_step_ls_all<%s, %d, false>" if lanes == 2 else "k_batch_step_all<%s, %d, false>") % (
            "float" if storage == "f32" else "__half", ty)
        out[storage] = {"fluid_mlups": round(mlups, 1), "ms_per_step": ms, "tile_y": ty, "lanes": lanes,
                        "speedup_vs_plain_loop": round(mlups / out["plain_loop_fluid_mlups"], 2),
                        "timed_steps_in_graphs": c1["graph_steps"] - c0["graph_steps"],
                        "instances_flagged": flags,
                        "roofline": roofline(kern, "k_batch_step_all_c4_64_instances.md", fluid, 0, storage, ms),
                        "error_vs_oracle": err_entry(*worst, storage, at_step=warm + steps,
                                                     nodes="all fluid nodes of instances 0, 3, 5 (improved, "
                                                           "Martys-Chen, LLKC)") if picks else None}
        if bars and picks:
            e = out[storage]["error_vs_oracle"]
            e["within_bar"] = bool(ok)
            e["bar"] = None
            e["bar_per_instance"] = {str(k): [float("%.3e" % v) for v in bars[k]] for k in picks}
            e["bar_rule"] = ("twice the error FP16 storage alone gives on the instance at this step: the FP64 "
                             "oracle with the same storage rounding after every step "
                             "(tests/golden/f16_model_c4.npz)")
    return out


# ----------------------------------------------------------------- served

def served_rows(M, torch, W, args):
    import numpy as np
    import oracle
    from paper_2009_12584_amd.serve import Request, percentile, serve, summarize

    oracle.build()
    n_req, chunk = args.served_requests, 200
    reqs = []
    for t, c in W.config5_requests(n=n_req):
        m = M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
        reqs.append(Request(t, m, c.rhoA0, c.rhoB0, c.steps, c.params(), tag=c.name))
    # the three requests of least work are also checked against the oracle
    work = sorted(reqs, key=lambda r: int((r.mask == 0).sum()) * r.steps)
    check = {r.tag: r for r in work[:3]}
    stream = torch.cuda.Stream()
    done, makespan = serve(reqs, hbm_budget=64 << 30, max_slots=64, chunk=chunk, stream=stream, diag_every=chunk,
                           keep_tags=set(check))
    s = summarize(done, makespan)
    worst = (0.0, 0.0)
    for d in done:
        if d.tag in check:
            r = check[d.tag]
            o = oracle.Oracle(r.mask, r.rhoA0, r.rhoB0, **r.params)
            o.step(r.steps)
            er, eu = errors(r.mask, d.fields, o.fields())
            worst = (max(worst[0], er), max(worst[1], eu))
    # the same requests one by one: each request's set-up, per-step time (over
    # up to 1000 steps in graphs of 100) and read-back are measured alone on
    # the device; its service time is set-up + steps x per-step + read-back,
    # and the first-come first-served queue of the same arrivals follows
    service, lu = [], 0
    for r in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim = M.Simulation(r.mask, r.rhoA0, r.rhoB0, stream=stream, graph_steps=100, diag_every=100, **r.params)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        n = min(r.steps, 1000)
        with Timer(torch, stream) as tm:
            sim.step(n)
        t1 = time.perf_counter()
        sim.fields()
        t_read = time.perf_counter() - t1
        sim.close()
        service.append(t_setup + tm.ms * 1e-3 / n * r.steps + t_read)
        lu += int((r.mask == 0).sum()) * r.steps
    plain = lu / sum(service) / 1e6
    by_arrival = sorted(zip(reqs, service), key=lambda rs: rs[0].arrival)

    def fifo(scale):
        free, lat = 0.0, []
        for r, sv in by_arrival:
            free = max(free, r.arrival * scale) + sv
            lat.append(free - r.arrival * scale)
        return lat

    lat = fifo(1.0)
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    s = rnd(s)
    s.update({"workload": "%d requests, Poisson 200/s (seed 12345), W in 64..2048, H in 64..1024, 2k-20k steps, "
                          "mixed BCs and angles, FP32; 64 slots admitted first-come first-served, chunks of %d "
                          "steps, fused diagnostics every %d launches" % (n_req, chunk, chunk),
              "roofline": {"bound": "hbm", "achieved": round(s["fluid_mlups"] * ALG_BYTES["f32"] / 1e3, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(s["fluid_mlups"] * ALG_BYTES["f32"] / 1e3 / HBM_PEAK_GBS, 4)},
              "error_vs_oracle": err_entry(*worst, "f32", nodes="all fluid nodes of the 3 least-work requests",
                                           at_step="each request's own step count"),
              "one_by_one_fluid_mlups": round(plain, 1), "speedup_vs_one_by_one": round(s["fluid_mlups"] / plain, 2),
              "one_by_one_fifo_model_p50_latency_s": round(percentile(lat, 50), 4),
              "one_by_one_fifo_model_p99_latency_s": round(percentile(lat, 99), 4),
              "one_by_one_note": "modelled: first-come first-served queue of the same arrivals over service times "
                                 "measured per request alone on the device"})
    # the same trace with its arrival times stretched so that requests arrive
    # at 80% of the rate the pool sustained above (still a Poisson process)
    rate = 0.8 * n_req / s["makespan_s"]
    scale = 200.0 / rate
    done3, mk3 = serve(reqs, hbm_budget=64 << 30, max_slots=64, chunk=chunk, stream=stream, time_scale=scale,
                       diag_every=chunk)
    s3 = rnd(summarize(done3, mk3))
    lat3 = fifo(scale)
    s3.update({"arrival_rate_per_s": round(rate, 3),
               "one_by_one_fifo_model_p50_latency_s": round(percentile(lat3, 50), 4),
               "one_by_one_fifo_model_p99_latency_s": round(percentile(lat3, 99), 4)})
    s["at_80pct_of_capacity"] = s3
    return s


# ----------------------------------------------------------------- CPU baseline

def cpu_baseline(M, W):
    """The FP64 oracle, as it stands, on the host: the headline workload on all
    threads and on one, and short samples of the other configurations."""
    import oracle

    oracle.build()
    allt = oracle.threads()

    def mlups(c, mask, steps, threads):
        oracle.set_threads(threads)
        o = oracle.Oracle(mask, c.rhoA0, c.rhoB0, **c.params())
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        return int((mask == 0).sum()) * steps / dt / 1e6, dt

    c3 = W.config3(0)
    g = c3.geometry
    m3 = oracle.mask_disk(c3.nx, c3.ny, g[1], g[2], g[3])
    v_all, dt_all = mlups(c3, m3, 600, allt)
    v_one, dt_one = mlups(c3, m3, 40, 1)
    samples = {}
    c1 = W.config1()
    samples["config1_full_2000_steps"] = round(mlups(c1, c1.mask_user, 2000, allt)[0], 2)
    c2 = W.config2()
    m2 = oracle.mask_plane(c2.nx, c2.ny, c2.geometry[1], c2.geometry[2])
    samples["config2_500_steps"] = round(mlups(c2, m2, 500, allt)[0], 2)
    c4 = W.config4_instances(64)[0]
    m4 = oracle.mask_plane(c4.nx, c4.ny, c4.geometry[1], c4.geometry[2])
    samples["config4_instance0_300_steps"] = round(mlups(c4, m4, 300, allt)[0], 2)
    r = W.roofline_case()
    samples["r5600x4000_mixture_2_steps"] = round(mlups(r, r.mask_user, 2, allt)[0], 2)
    oracle.set_threads(allt)
    return {"value": round(v_all, 2), "unit": "MLUPS", "cores": allt, "kind": "oracle",
            "sample": "configuration 3 (1024x1024 disk, improved scheme), 600 steps of the FP64 C oracle on %d "
                      "threads (%.1f s)" % (allt, dt_all),
            "single_thread": {"value": round(v_one, 2), "sample": "40 steps on 1 thread (%.1f s)" % dt_one},
            "other_configs_mlups_all_threads": samples,
            "host": {"cpu": oracle.host_cpu(), "nproc": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
                     "build": " ".join(oracle.FLAGS)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=49800,
                    help="timed steps of the headline (configuration 3); with the default warmup the run is the "
                         "configuration's 50,000 steps")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--large-steps", type=int, default=200, help="timed steps of each 5600x4000 row")
    ap.add_argument("--large-only", default="",
                    help="comma list of 5600x4000 rows to run (e.g. plane30_mc_f32); default all")
    ap.add_argument("--config2-steps", type=int, default=19800,
                    help="timed steps of configuration 2 (after 200 untimed: the run ends at its 20,000 steps)")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--served-requests", type=int, default=400)
    ap.add_argument("--rows", default="headline,large,config2,batched,served,cpu",
                    help="comma list of rows to run (profiling runs select one)")
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="steps per captured HIP graph (0 = plain launches only, which per-dispatch counter "
                         "collection needs); default min(100, steps)")
    ap.add_argument("--fixed-shapes", action="store_true",
                    help="fixed launch shapes for the batched row instead of the autotuner (counter runs name one "
                         "kernel)")
    ap.add_argument("--autotune-shapes", action="store_true",
                    help="pick the launch shapes of configurations 3 and 2 with the autotuner instead of the fixed "
                         "64 x 8, one lane per node")
    ap.add_argument("--no-oracle", action="store_true",
                    help="no oracle comparisons (error_vs_oracle null) and no untimed run to 50,000 steps: for "
                         "profiler runs, which time kernels only")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the slab decomposition is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    import paper_2009_12584_amd as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    rows = set(args.rows.split(","))
    probe = copy_probe(torch)
    if "headline" in rows:
        out = headline(M, torch, W, args, probe)
    else:
        out = {"metric": METRIC, "value": None, "unit": "MLUPS", "n_gpus": 1, "steps": 0, "warmup": 0,
               "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32", "data": "synthetic", "config": {"workload": "headline row skipped (--rows)"},
               "copy_probe": probe}
    print("bench: headline done", file=sys.stderr, flush=True)
    if "large" in rows:
        out["rows_5600x4000"] = rows_5600x4000(M, torch, W, args, probe)
        print("bench: 5600x4000 rows done", file=sys.stderr, flush=True)
    if "config2" in rows:
        out["config2"] = config2_row(M, torch, W, args)
    if "batched" in rows:
        out["batched"] = batched_rows(M, torch, W, args)
        print("bench: batched rows done", file=sys.stderr, flush=True)
    if "served" in rows:
        out["served"] = served_rows(M, torch, W, args)
        print("bench: served rows done", file=sys.stderr, flush=True)
    if "cpu" in rows:
        out["cpu_baseline"] = cpu_baseline(M, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
