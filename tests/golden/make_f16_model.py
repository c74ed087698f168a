"""Writes the error that FP16 population storage alone produces against the
FP64 oracle, on the instances the batched FP16 tests and bench row check.

Calls only ``oracle`` (the FP64 oracle and its storage model) and
``workloads`` (the seeded inputs): no value here comes from the HIP library.
For each of instances 0, 3 and 5 of the 64-instance batch (improved scheme,
Martys-Chen, LLKC) it runs the plain oracle and the oracle with the FP16
storage rounding side by side and stores, at each checkpoint, the largest
relative density error over both components and the largest absolute
velocity error over fluid nodes, with a hash of the instance's inputs.  The
FP16 tolerance of those tests is twice these values.  Run from the
repository root (about 4 minutes on 8 cores):

    python tests/golden/make_f16_model.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.storage_model import StorageModel  # noqa: E402
import workloads as W  # noqa: E402

INSTANCES = (0, 3, 5)
CHECKPOINTS = (10, 100, 300, 600, 1100, 2100)


def errors(mask, got, ref):
    fl = mask == 0
    er = max(float(np.max(np.abs(got[k] - ref[k])[fl] / ref[k][fl])) for k in (0, 1))
    eu = max(float(np.max(np.abs(got[k] - ref[k])[fl])) for k in (2, 3))
    return er, eu


def main():
    oracle.build()
    cases = W.config4_instances(64)
    out = {"instances": np.array(INSTANCES), "steps": np.array(CHECKPOINTS)}
    er_all = np.zeros((len(INSTANCES), len(CHECKPOINTS)))
    eu_all = np.zeros_like(er_all)
    for a, k in enumerate(INSTANCES):
        c = cases[k]
        m = oracle.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2])
        exact = oracle.Oracle(m, c.rhoA0, c.rhoB0, **c.params())
        model = StorageModel(m, c.rhoA0, c.rhoB0, **c.params())
        for b, T in enumerate(CHECKPOINTS):
            exact.step(T - exact.t)
            model.step(T - model.t)
            er_all[a, b], eu_all[a, b] = errors(m, model.fields(), exact.fields())
            print(c.name, T, "%.3e %.3e" % (er_all[a, b], eu_all[a, b]), flush=True)
        out["input_sha_%d" % k] = np.array(W.input_hash(c, m))
    out["err_rho"] = er_all
    out["err_u"] = eu_all
    np.savez_compressed(os.path.join(HERE, "f16_model_c4.npz"), **out)


if __name__ == "__main__":
    main()
