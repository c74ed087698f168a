"""FP64 CPU oracle for the two-component pseudopotential LBM with wetting walls.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path (the HIP library and
its binding) never imports this package, and this package imports nothing
from the product.

The arithmetic lives in ``lbm_oracle.c`` (plain C, IEEE double, no FMA
contraction); this module only builds it with gcc and marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_MARTYS_CHEN, BC_LLKC, BC_IMPROVED, BC_FIXED_VIRTUAL = 0, 1, 2, 3
AVG_D2Q25, AVG_D2Q9 = 0, 1
MODEL_TWO, MODEL_SC1 = 0, 1


# -march=native for the host that runs it; no contraction and no fast-math,
# so every IEEE double operation rounds exactly as written, on any CPU
FLAGS = ["-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-Wall"]


def host_cpu() -> str:
    """CPU model of this host (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _stamp() -> str:
    return host_cpu() + "|" + " ".join(FLAGS)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc for this host's CPU.  A library built on
    another CPU model (the stamp file beside it) or older than its sources is
    rebuilt."""
    stamp_file = _LIB + ".host"
    stale = (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "lbm_oracle.h"))))
    if not stale:
        try:
            stale = open(stamp_file).read() != _stamp()
        except OSError:
            stale = True
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *FLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
        with open(stamp_file, "w") as f:
            f.write(_stamp())
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("periodic", ctypes.c_uint),
        ("tau", ctypes.c_double), ("G", ctypes.c_double), ("bc", ctypes.c_int),
        ("Gw", ctypes.c_double), ("chiA", ctypes.c_double), ("chiB", ctypes.c_double),
        ("avg", ctypes.c_int), ("model", ctypes.c_int), ("rho0", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        L.ora_create.argtypes = [ctypes.POINTER(_Params), P, P, P, ctypes.POINTER(P)]
        L.ora_create.restype = I
        L.ora_destroy.argtypes = [P]
        L.ora_step.argtypes = [P, ctypes.c_long]
        L.ora_step.restype = I
        L.ora_time.argtypes = [P]
        L.ora_time.restype = ctypes.c_long
        for name in ("ora_fields", "ora_forces"):
            getattr(L, name).argtypes = [P, P, P, P, P]
        L.ora_virtual_density.argtypes = [P, P, P]
        L.ora_get_populations.argtypes = [P, P]
        L.ora_set_populations.argtypes = [P, P]
        L.ora_totals.argtypes = [P, P]
        L.ora_mask_plane.argtypes = [I, I, D, D, I, P]
        L.ora_mask_disk.argtypes = [I, I, D, D, D, I, P]
        L.ora_classify.argtypes = [I, I, ctypes.c_uint, P, P, P]
        L.ora_lattice.argtypes = [P] * 7
        L.ora_equilibrium.argtypes = [D, D, D, P]
        L.ora_guo_source.argtypes = [D, D, D, D, D, P]
        L.ora_threads.restype = I
        L.ora_set_threads.argtypes = [I]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def threads() -> int:
    return int(lib().ora_threads())


def set_threads(n: int) -> None:
    """Threads of the following oracle calls in this process."""
    lib().ora_set_threads(int(n))


def lattice():
    """D2Q9 weights/velocities/opposites and the D2Q25 averaging table."""
    w9 = np.zeros(9)
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    opp = np.zeros(9, np.int32)
    w25 = np.zeros(24)
    ex = np.zeros(24, np.int32)
    ey = np.zeros(24, np.int32)
    lib().ora_lattice(*[_ptr(a) for a in (w9, cx, cy, opp, w25, ex, ey)])
    return dict(w9=w9, cx=cx, cy=cy, opp=opp, w25=w25, ex=ex, ey=ey)


def equilibrium(rho, ux, uy):
    out = np.zeros(9)
    lib().ora_equilibrium(rho, ux, uy, _ptr(out))
    return out


def guo_source(tau, ux, uy, Fx, Fy):
    out = np.zeros(9)
    lib().ora_guo_source(tau, ux, uy, Fx, Fy, _ptr(out))
    return out


def mask_plane(nx, ny, beta, R0, borders=True):
    out = np.zeros((ny, nx), np.uint8)
    lib().ora_mask_plane(nx, ny, float(beta), float(R0), int(bool(borders)), _ptr(out))
    return out


def mask_disk(nx, ny, cx, cy, R, borders=True):
    out = np.zeros((ny, nx), np.uint8)
    lib().ora_mask_disk(nx, ny, float(cx), float(cy), float(R), int(bool(borders)), _ptr(out))
    return out


def classify(mask, periodic):
    mask = np.ascontiguousarray(mask, np.uint8)
    ny, nx = mask.shape
    nbr = np.zeros((ny, nx), np.uint8)
    cls = np.zeros((ny, nx), np.uint8)
    lib().ora_classify(nx, ny, int(periodic), _ptr(mask), _ptr(nbr), _ptr(cls))
    return nbr, cls


class Oracle:
    """One simulation held by the C oracle (populations in FP64)."""

    def __init__(self, mask, rhoA0, rhoB0, *, tau, G, bc, Gw=0.0, chiA=1.0, chiB=1.0,
                 avg=AVG_D2Q25, periodic=0, model=MODEL_TWO, rho0=1.0):
        """rhoB0 may be None for the single-component model (model=MODEL_SC1)."""
        mask = np.ascontiguousarray(mask, np.uint8)
        self.ny, self.nx = mask.shape
        self.mask = mask
        rA = np.ascontiguousarray(rhoA0, np.float64).reshape(self.ny, self.nx)
        rB = np.zeros_like(rA) if rhoB0 is None else np.ascontiguousarray(rhoB0, np.float64).reshape(self.ny, self.nx)
        p = _Params(self.nx, self.ny, int(periodic), float(tau), float(G), int(bc), float(Gw),
                    float(chiA), float(chiB), int(avg), int(model), float(rho0))
        h = ctypes.c_void_p()
        rc = lib().ora_create(ctypes.byref(p), _ptr(mask), _ptr(rA), _ptr(rB), ctypes.byref(h))
        if rc != 0:
            raise ValueError("ora_create rejected the inputs (code %d)" % rc)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().ora_destroy(h)
            self._h = None

    @property
    def t(self) -> int:
        return int(lib().ora_time(self._h))

    def step(self, n: int = 1):
        rc = lib().ora_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError("ora_step failed (%d)" % rc)

    def _grid(self, k):
        return [np.zeros((self.ny, self.nx)) for _ in range(k)]

    def fields(self):
        """(rhoA, rhoB, ux, uy) at the current time."""
        a = self._grid(4)
        lib().ora_fields(self._h, *[_ptr(x) for x in a])
        return tuple(a)

    def forces(self):
        """(FAx, FAy, FBx, FBy): total force per component at the current time."""
        a = self._grid(4)
        lib().ora_forces(self._h, *[_ptr(x) for x in a])
        return tuple(a)

    def virtual_density(self):
        a = self._grid(2)
        lib().ora_virtual_density(self._h, *[_ptr(x) for x in a])
        return tuple(a)

    def populations(self):
        out = np.zeros((2, 9, self.ny, self.nx))
        lib().ora_get_populations(self._h, _ptr(out))
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(2, 9, self.ny, self.nx)
        lib().ora_set_populations(self._h, _ptr(f))

    def totals(self):
        """(mass A, mass B, momentum x, momentum y) summed over fluid nodes."""
        out = np.zeros(4)
        lib().ora_totals(self._h, _ptr(out))
        return out
