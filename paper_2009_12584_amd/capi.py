"""ctypes declarations of the libmclbm.so C ABI (include/mclbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmclbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EAGAIN, LBM_EDEVICE, LBM_ENUMERIC, LBM_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
BC_MARTYS_CHEN, BC_LLKC, BC_VIRTUAL_IMPROVED, BC_FIXED_VIRTUAL = 0, 1, 2, 3
AVG_D2Q25, AVG_D2Q9 = 0, 1
STORE_F32, STORE_F16 = 0, 1
MODEL_TWO, MODEL_SC1 = 0, 1

# every symbol include/mclbm.h declares
EXPORTS = [
    "lbm_params_default", "lbm_create", "lbm_step", "lbm_time", "lbm_launch_counts", "lbm_fields", "lbm_fields_device",
    "lbm_forces", "lbm_diag", "lbm_classify", "lbm_state_bytes", "lbm_get_state", "lbm_set_state",
    "lbm_destroy", "lbm_strerror", "lbm_last_error", "lbm_mask_plane", "lbm_mask_disk", "lbm_copy_probe",
    "lbm_contour_fit", "lbm_batch_contour_fit", "lbm_line_probe",
    "lbm_params_state_bytes", "lbm_batch_create", "lbm_batch_step", "lbm_batch_launch_counts", "lbm_batch_fields",
    "lbm_batch_diag", "lbm_batch_get_state", "lbm_batch_set_state", "lbm_batch_fluid_nodes", "lbm_batch_destroy",
    "lbm_pool_create", "lbm_pool_footprint", "lbm_pool_admit", "lbm_pool_admit_noalloc", "lbm_pool_advance", "lbm_pool_poll",
    "lbm_pool_status", "lbm_pool_fields", "lbm_pool_diag", "lbm_pool_get_state", "lbm_pool_set_state", "lbm_pool_release",
    "lbm_pool_stats", "lbm_pool_progress", "lbm_pool_destroy",
]


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("periodic", ctypes.c_uint32),
        ("tau", ctypes.c_double), ("G", ctypes.c_double), ("bc", ctypes.c_int32),
        ("G_w", ctypes.c_double), ("chi", ctypes.c_double * 2), ("avg", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("rho_ref", ctypes.c_double * 2), ("diag_every", ctypes.c_int32),
        ("drift_tol", ctypes.c_double), ("graph_steps", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("model", ctypes.c_int32), ("psi_rho0", ctypes.c_double), ("lanes", ctypes.c_int32),
    ]


class LbmDiag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * 2), ("mass0", ctypes.c_double * 2), ("momentum", ctypes.c_double * 2),
        ("max_speed", ctypes.c_double), ("step", ctypes.c_int64), ("flags", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class LbmContourReq(ctypes.Structure):
    _fields_ = [("level", ctypes.c_double), ("skip", ctypes.c_int32), ("roi", ctypes.c_int32 * 4)]


class LbmCircle(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xc", ctypes.c_double), ("yc", ctypes.c_double), ("R", ctypes.c_double),
                ("rms", ctypes.c_double), ("max_dev", ctypes.c_double)]


class LbmError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__("%s (%d): %s" % (_strerror(code), code, detail))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmclbm.so is not built: run __graft_entry__.build() "
                              "(or python -m paper_2009_12584_amd._build)")
        # torch ships its own HIP and HSA runtimes: loading them first makes this
        # library bind to the same ones (one runtime per process); the other
        # order leaves torch without devices.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        PP = ctypes.POINTER(LbmParams)
        sig = {
            "lbm_params_default": (None, [PP]),
            "lbm_create": (I32, [PP, P, P, P, P, ctypes.POINTER(P)]),
            "lbm_step": (I32, [P, I64]),
            "lbm_time": (I64, [P]),
            "lbm_launch_counts": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
            "lbm_fields": (I32, [P, P, P, P, P]),
            "lbm_fields_device": (I32, [P, P, P, P, P]),
            "lbm_forces": (I32, [P, P, P, P, P, P, P]),
            "lbm_diag": (I32, [P, ctypes.POINTER(LbmDiag)]),
            "lbm_classify": (I32, [P, P, P]),
            "lbm_state_bytes": (SZ, [P]),
            "lbm_get_state": (I32, [P, P, ctypes.POINTER(I64)]),
            "lbm_set_state": (I32, [P, P, I64]),
            "lbm_destroy": (I32, [P]),
            "lbm_strerror": (ctypes.c_char_p, [I32]),
            "lbm_last_error": (ctypes.c_char_p, [P]),
            "lbm_mask_plane": (I32, [I32, I32, D, D, I32, P]),
            "lbm_mask_disk": (I32, [I32, I32, D, D, D, I32, P]),
            "lbm_copy_probe": (I32, [P, P, SZ, P]),
            "lbm_contour_fit": (I32, [P, ctypes.POINTER(LbmContourReq), ctypes.POINTER(LbmCircle)]),
            "lbm_batch_contour_fit": (I32, [P, I32, ctypes.POINTER(LbmContourReq), ctypes.POINTER(LbmCircle)]),
            "lbm_line_probe": (I32, [P, I32, I32, I32, I32, I32, D, P]),
            "lbm_params_state_bytes": (SZ, [PP]),
            "lbm_batch_create": (I32, [I32, PP, P, P, P, P, I32, ctypes.POINTER(P)]),
            "lbm_batch_step": (I32, [P, I64]),
            "lbm_batch_launch_counts": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
            "lbm_batch_get_state": (I32, [P, I32, P]),
            "lbm_batch_set_state": (I32, [P, I32, P]),
            "lbm_batch_fields": (I32, [P, I32, P, P, P, P]),
            "lbm_batch_diag": (I32, [P, I32, ctypes.POINTER(LbmDiag)]),
            "lbm_batch_fluid_nodes": (I64, [P]),
            "lbm_batch_destroy": (I32, [P]),
            "lbm_pool_create": (I32, [SZ, I32, I32, I32, P, ctypes.POINTER(P)]),
            "lbm_pool_footprint": (SZ, [PP]),
            "lbm_pool_admit": (I32, [P, PP, P, P, P, I64, ctypes.POINTER(I32)]),
            "lbm_pool_admit_noalloc": (I32, [P, PP, P, P, P, I64, ctypes.POINTER(I32)]),
            "lbm_pool_advance": (I32, [P, I64]),
            "lbm_pool_poll": (I32, [P, P, I32, ctypes.POINTER(I32)]),
            "lbm_pool_fields": (I32, [P, I32, P, P, P, P]),
            "lbm_pool_diag": (I32, [P, I32, ctypes.POINTER(LbmDiag)]),
            "lbm_pool_status": (I32, [P, I32]),
            "lbm_pool_get_state": (I32, [P, I32, P]),
            "lbm_pool_set_state": (I32, [P, I32, P]),
            "lbm_pool_release": (I32, [P, I32]),
            "lbm_pool_stats": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(SZ)]),
            "lbm_pool_progress": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]),
            "lbm_pool_destroy": (I32, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().lbm_strerror(code).decode()
    except Exception:  # library unavailable while reporting
        return "error"


def check(code, handle=None):
    if code != LBM_OK:
        detail = lib().lbm_last_error(handle).decode(errors="replace")
        raise LbmError(code, detail)
    return code


def make_params(nx, ny, *, tau=1.0, G=0.9, bc=BC_MARTYS_CHEN, Gw=0.0, chiA=1.0, chiB=1.0, avg=AVG_D2Q25,
                periodic=0, storage=STORE_F32, rho_ref=None, diag_every=0, drift_tol=0.0, graph_steps=0,
                tile_y=0, model=MODEL_TWO, rho0=1.0, lanes=0) -> LbmParams:
    p = LbmParams()
    lib().lbm_params_default(ctypes.byref(p))
    p.nx, p.ny, p.periodic = int(nx), int(ny), int(periodic)
    p.tau, p.G, p.bc, p.G_w = float(tau), float(G), int(bc), float(Gw)
    p.chi[0], p.chi[1] = float(chiA), float(chiB)
    p.avg = int(avg)
    p.storage = STORE_F16 if storage in ("f16", STORE_F16) else STORE_F32
    rr = (math.nan, math.nan) if rho_ref is None else rho_ref
    p.rho_ref[0], p.rho_ref[1] = float(rr[0]), float(rr[1])
    p.diag_every, p.drift_tol = int(diag_every), float(drift_tol)
    p.graph_steps, p.tile_y = int(graph_steps), int(tile_y)
    p.model, p.psi_rho0, p.lanes = int(model), float(rho0), int(lanes)
    return p


def make_contour_req(level=0.5, skip=3, roi=None) -> LbmContourReq:
    """roi = (x0, y0, x1, y1) inclusive, or None for the whole grid."""
    q = LbmContourReq()
    q.level, q.skip = float(level), int(skip)
    for k, v in enumerate(roi if roi is not None else (0, 0, 0, 0)):
        q.roi[k] = int(v)
    return q
