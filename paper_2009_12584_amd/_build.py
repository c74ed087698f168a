"""Builds libmclbm.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmclbm.so")
SOURCES = ["lbm_single.hip", "lbm_step_f32.hip", "lbm_step_f16.hip", "lbm_batch.hip", "lbm_batch_f32.hip",
           "lbm_batch_f16.hip", "lbm_analysis.hip"]
HEADERS = ["lbm_tiling.hpp", "lbm_plan.hpp", "lbm_device.hpp", "lbm_pair.hpp", "lbm_sc1.hpp", "lbm_common.hpp", "lbm_step_kernels.hpp", "lbm_batch_kernels.hpp", "lbm_analysis.hpp"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libmclbm.so (always recompiles)."""
    objs, procs = [], []
    for src in sources():  # translation units compile in parallel
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = ["hipcc", *[f for f in FLAGS if f != "-shared"], "-c", "-o", obj, src]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        objs.append(obj)
    for src, p in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
        if verbose and err:
            print(err)
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
