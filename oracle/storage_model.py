"""Reduced-precision population storage applied to the FP64 oracle.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests and the
benchmark's error bars use it; the product path never imports it.

The GPU library keeps each step's post-collision populations in storage of
lower precision than its FP32 arithmetic.  With FP16 storage a node's eight
moving populations of component sigma are kept as the deviation
d_i = f_i - w_i rho_ref^sigma, scaled by 2^10 and rounded to the nearest
FP16 value, and its rest population in FP32 as the remainder that keeps the
node's mass: d_0 + sum_i (d_i - round(d_i)), rounded once to FP32.  That
storage rounding is the whole difference between the FP16 path and exact
arithmetic at first order, so its effect on a trajectory is a property of the
format, not of the kernels: this module re-applies it to the oracle's state
after every oracle step and so gives the error that FP16 storage alone
produces on a workload, from which the tolerance of the FP16 tests and bench
rows is derived.

The oracle streams by push with half-way bounce-back, so its state after a
step holds the populations at their destination.  ``origin_maps`` inverts
that: the population in direction i at fluid node y came from node y - c_i in
direction i, or, when y - c_i is solid, from y itself in the opposite
direction (bounce-back, Section 2).  Each post-collision population of a fluid
node lands in exactly one place, so the map is a bijection on fluid nodes:
the state is mapped back to its nodes of origin, rounded there as the storage
rounds it, and mapped forward again.
"""
from __future__ import annotations

import numpy as np

from . import Oracle, lattice

FP16_SCALE = 1024.0


def default_rho_ref(mask, rhoA0, rhoB0):
    """The library's default deviation references: per component, the
    smallest initial density over fluid nodes."""
    fl = np.asarray(mask) == 0
    return (float(np.asarray(rhoA0)[fl].min()), float(np.asarray(rhoB0)[fl].min()))


def origin_maps(mask, periodic):
    """Per direction i: (destination fluid nodes y, origin nodes, origin
    directions), flat indices.  Neighbours wrap in periodic directions; fluid
    never sits on a non-periodic border, so its neighbours stay inside."""
    L = lattice()
    cx, cy, opp = L["cx"], L["cy"], L["opp"]
    mask = np.asarray(mask)
    ny, nx = mask.shape
    Y, X = np.mgrid[0:ny, 0:nx]
    flat = mask.ravel()
    dest = np.nonzero(flat == 0)[0]
    maps = []
    for i in range(9):
        sx = (X - cx[i]) % nx if periodic & 1 else X - cx[i]
        sy = (Y - cy[i]) % ny if periodic & 2 else Y - cy[i]
        src = (sy * nx + sx).ravel()[dest]
        solid = flat[src] != 0
        maps.append((dest, np.where(solid, dest, src), np.where(solid, opp[i], i)))
    return maps


def to_origin(F, maps):
    """Post-streaming populations (2, 9, n) -> post-collision ones at their
    nodes of origin (solid nodes stay 0)."""
    Q = np.zeros_like(F)
    for i, (dest, src, sdir) in enumerate(maps):
        for c in range(F.shape[0]):
            Q[c, sdir, src] = F[c, i, dest]
    return Q


def from_origin(Q, maps):
    """The inverse of ``to_origin``: streaming with half-way bounce-back."""
    F = np.zeros_like(Q)
    for i, (dest, src, sdir) in enumerate(maps):
        for c in range(Q.shape[0]):
            F[c, i, dest] = Q[c, sdir, src]
    return F


def round_fp16_storage(Q, fluid, rho_ref, scale=FP16_SCALE):
    """Post-collision populations Q (2, 9, n) as FP16 storage keeps them:
    moving deviations rounded to FP16 after scaling, rest deviation the FP32
    remainder of the node's mass."""
    w = lattice()["w9"]
    out = Q.copy()
    for c in range(Q.shape[0]):
        q = Q[c][:, fluid]
        dev = q - w[:, None] * rho_ref[c]
        kept = (dev[1:] * scale).astype(np.float16).astype(np.float64) / scale
        rest = (dev[0] + (dev[1:] - kept).sum(axis=0)).astype(np.float32).astype(np.float64)
        out[c][0, fluid] = rest + w[0] * rho_ref[c]
        out[c][1:, fluid] = kept + w[1:, None] * rho_ref[c]
    return out


class StorageModel:
    """The FP64 oracle with the FP16 storage rounding applied after every
    step (two-component model)."""

    def __init__(self, mask, rhoA0, rhoB0, *, rho_ref=None, **params):
        self.mask = np.ascontiguousarray(mask, np.uint8)
        self.o = Oracle(self.mask, rhoA0, rhoB0, **params)
        self.rho_ref = rho_ref if rho_ref is not None else default_rho_ref(self.mask, rhoA0, rhoB0)
        self.maps = origin_maps(self.mask, int(params.get("periodic", 0)))
        self.fluid = self.mask.ravel() == 0
        self.shape = self.mask.shape

    @property
    def t(self):
        return self.o.t

    def step(self, n=1):
        ny, nx = self.shape
        for _ in range(int(n)):
            self.o.step(1)
            F = self.o.populations().reshape(2, 9, nx * ny)
            Q = round_fp16_storage(to_origin(F, self.maps), self.fluid, self.rho_ref)
            self.o.set_populations(from_origin(Q, self.maps).reshape(2, 9, ny, nx))

    def fields(self):
        return self.o.fields()

    def totals(self):
        return self.o.totals()
