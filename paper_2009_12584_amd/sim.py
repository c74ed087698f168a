"""Python handles over the C ABI: one simulation, a batch, a serving pool.

PyTorch is used only for device memory and streams (a stream handle, device
pointers); numpy carries host arrays across the ABI.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import capi
from .capi import check, lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _host(a, dtype, shape):
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


def _diag_dict(d) -> dict:
    return dict(mass=(d.mass[0], d.mass[1]), mass0=(d.mass0[0], d.mass0[1]),
                momentum=(d.momentum[0], d.momentum[1]), max_speed=d.max_speed, step=d.step, flags=d.flags)


def _checked(code, handle=None, raise_on_flags=True):
    """check(), except that LBM_ENUMERIC may be returned instead of raised."""
    if code == capi.LBM_ENUMERIC and not raise_on_flags:
        return code
    return check(code, handle)


def state_bytes(nx, ny, storage="f32", **prm) -> int:
    """Bytes of one simulation's raw state (lbm_params_state_bytes)."""
    p = capi.make_params(nx, ny, storage=storage, **prm)
    return int(lib().lbm_params_state_bytes(ctypes.byref(p)))


def _circle(c) -> dict:
    return dict(n=int(c.n), xc=c.xc, yc=c.yc, R=c.R, rms=c.rms, max_dev=c.max_dev)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)  # a torch.cuda.Stream


def mask_plane(nx, ny, beta, R0, borders=True) -> np.ndarray:
    """Plane wall of Section 3.1, rasterised on the device (bit-exact FP64)."""
    out = np.zeros((ny, nx), np.uint8)
    check(lib().lbm_mask_plane(int(nx), int(ny), float(beta), float(R0), int(bool(borders)), _p(out)))
    return out


def mask_disk(nx, ny, cx, cy, R, borders=True) -> np.ndarray:
    """Disk wall of Section 4, rasterised on the device."""
    out = np.zeros((ny, nx), np.uint8)
    check(lib().lbm_mask_disk(int(nx), int(ny), float(cx), float(cy), float(R), int(bool(borders)), _p(out)))
    return out


class Simulation:
    """One two-component simulation resident on the GPU (lbm_create ... lbm_destroy)."""

    def __init__(self, mask, rhoA0, rhoB0, *, stream=None, **params):
        mask = np.ascontiguousarray(mask, np.uint8)
        self.ny, self.nx = mask.shape
        self.params = capi.make_params(self.nx, self.ny, **params)
        rA = _host(rhoA0, np.float64, mask.shape)
        # the single-component model reads no rhoB0
        rB = None if rhoB0 is None else _host(rhoB0, np.float64, mask.shape)
        h = ctypes.c_void_p()
        code = lib().lbm_create(ctypes.byref(self.params), _p(mask), _p(rA), None if rB is None else _p(rB),
                                _stream_handle(stream), ctypes.byref(h))
        check(code)
        self._h = h

    # -- lifecycle
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lbm_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- stepping and outputs
    @property
    def t(self) -> int:
        return int(lib().lbm_time(self._h))

    def step(self, n: int = 1):
        check(lib().lbm_step(self._h, int(n)), self._h)

    def launch_counts(self) -> dict:
        """Steps run so far by graph replays and by plain launches."""
        g, p = ctypes.c_int64(), ctypes.c_int64()
        check(lib().lbm_launch_counts(self._h, ctypes.byref(g), ctypes.byref(p)), self._h)
        return {"graph_steps": int(g.value), "plain_steps": int(p.value)}

    def _grids(self, k):
        return [np.zeros((self.ny, self.nx)) for _ in range(k)]

    def fields(self):
        """(rhoA, rhoB, ux, uy) at the current time, float64 host arrays."""
        a = self._grids(4)
        check(lib().lbm_fields(self._h, *[_p(x) for x in a]), self._h)
        return tuple(a)

    def fields_device(self, rhoA, rhoB, ux, uy):
        """Writes the fields into float32 device tensors (or raw pointers) on the handle's stream."""
        ptrs = [ctypes.c_void_p(t if isinstance(t, int) else t.data_ptr()) if t is not None else None
                for t in (rhoA, rhoB, ux, uy)]
        check(lib().lbm_fields_device(self._h, *ptrs), self._h)

    def forces(self):
        """(FAx, FAy, FBx, FBy, rtA, rtB) at the current time."""
        a = self._grids(6)
        check(lib().lbm_forces(self._h, *[_p(x) for x in a]), self._h)
        return tuple(a)

    def diag(self, raise_on_flags=True) -> dict:
        d = capi.LbmDiag()
        _checked(lib().lbm_diag(self._h, ctypes.byref(d)), self._h, raise_on_flags)
        return _diag_dict(d)

    def contour_fit(self, level=0.5, skip=3, roi=None) -> dict:
        """Circle through the interface rho^A = level (lbm_contour_fit)."""
        c = capi.LbmCircle()
        q = capi.make_contour_req(level, skip, roi)
        check(lib().lbm_contour_fit(self._h, ctypes.byref(q), ctypes.byref(c)), self._h)
        return _circle(c)

    def line_probe(self, x0, y0, dx, dy, length, level, out):
        """Enqueues the interface crossing along a lattice line into the device
        double at `out` (an integer address, e.g. tensor.data_ptr() + 8 k)."""
        check(lib().lbm_line_probe(self._h, int(x0), int(y0), int(dx), int(dy), int(length), float(level),
                                   ctypes.c_void_p(int(out))), self._h)

    def classify(self):
        nbr = np.zeros((self.ny, self.nx), np.uint8)
        cls = np.zeros((self.ny, self.nx), np.uint8)
        check(lib().lbm_classify(self._h, _p(nbr), _p(cls)), self._h)
        return nbr, cls

    def get_state(self):
        n = int(lib().lbm_state_bytes(self._h))
        buf = np.zeros(n, np.uint8)
        step = ctypes.c_int64()
        check(lib().lbm_get_state(self._h, _p(buf), ctypes.byref(step)), self._h)
        return buf, int(step.value)

    def set_state(self, buf, step):
        buf = np.ascontiguousarray(buf, np.uint8)
        check(lib().lbm_set_state(self._h, _p(buf), int(step)), self._h)


class Batch:
    """Many simulations advanced by one launch per step (lbm_batch_*)."""

    def __init__(self, cases, *, storage="f32", graph_steps=0, tile_y=0, lanes=0, stream=None):
        """cases: iterable of (mask, rhoA0, rhoB0, params dict)."""
        cases = list(cases)
        n = len(cases)
        self.n = n
        self._keep = []
        P = (capi.LbmParams * n)()
        masks = (ctypes.c_void_p * n)()
        ras = (ctypes.c_void_p * n)()
        rbs = (ctypes.c_void_p * n)()
        self.shapes = []
        for k, (mask, rA, rB, prm) in enumerate(cases):
            mask = np.ascontiguousarray(mask, np.uint8)
            ny, nx = mask.shape
            rA = _host(rA, np.float64, mask.shape)
            rB = _host(rB, np.float64, mask.shape)
            self._keep += [mask, rA, rB]
            P[k] = capi.make_params(nx, ny, storage=storage, tile_y=tile_y, lanes=lanes, **prm)
            masks[k], ras[k], rbs[k] = mask.ctypes.data, rA.ctypes.data, rB.ctypes.data
            self.shapes.append((ny, nx))
        self._state_bytes = [int(lib().lbm_params_state_bytes(ctypes.byref(P[k]))) for k in range(n)]
        h = ctypes.c_void_p()
        check(lib().lbm_batch_create(n, P, masks, ras, rbs, _stream_handle(stream), int(graph_steps),
                                     ctypes.byref(h)))
        self._h = h
        self._keep = []

    @property
    def fluid_nodes(self) -> int:
        return int(lib().lbm_batch_fluid_nodes(self._h))

    def step(self, n=1):
        check(lib().lbm_batch_step(self._h, int(n)))

    def launch_counts(self) -> dict:
        """Steps run so far by graph replays and by plain launches."""
        g, p = ctypes.c_int64(), ctypes.c_int64()
        check(lib().lbm_batch_launch_counts(self._h, ctypes.byref(g), ctypes.byref(p)))
        return {"graph_steps": int(g.value), "plain_steps": int(p.value)}

    def fields(self, idx, which=(True, True, True, True), raise_on_flags=True):
        """(rhoA, rhoB, ux, uy) of instance idx; entries not in `which` are None."""
        ny, nx = self.shapes[idx]
        a = [np.zeros((ny, nx)) if w else None for w in which]
        _checked(lib().lbm_batch_fields(self._h, int(idx), *[_p(x) if x is not None else None for x in a]),
                 raise_on_flags=raise_on_flags)
        return tuple(a)

    def diag(self, idx, raise_on_flags=True):
        d = capi.LbmDiag()
        _checked(lib().lbm_batch_diag(self._h, int(idx), ctypes.byref(d)), raise_on_flags=raise_on_flags)
        return _diag_dict(d)

    def get_state(self, idx):
        ny, nx = self.shapes[idx]
        buf = np.zeros(self._state_bytes[idx], np.uint8)
        check(lib().lbm_batch_get_state(self._h, int(idx), _p(buf)))
        return buf

    def set_state(self, idx, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        assert buf.size == self._state_bytes[idx]
        check(lib().lbm_batch_set_state(self._h, int(idx), _p(buf)))

    def contour_fit(self, idx, level=0.5, skip=3, roi=None) -> dict:
        c = capi.LbmCircle()
        q = capi.make_contour_req(level, skip, roi)
        check(lib().lbm_batch_contour_fit(self._h, int(idx), ctypes.byref(q), ctypes.byref(c)))
        return _circle(c)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lbm_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """Resident slots with continuous batching (lbm_pool_*)."""

    def __init__(self, hbm_budget, max_slots, *, storage="f32", diag_every=0, stream=None):
        h = ctypes.c_void_p()
        st = capi.STORE_F16 if storage in ("f16", capi.STORE_F16) else capi.STORE_F32
        self.storage = st
        check(lib().lbm_pool_create(int(hbm_budget), int(max_slots), st, int(diag_every), _stream_handle(stream),
                                    ctypes.byref(h)))
        self._h = h
        self.shapes = {}
        self._state_bytes = {}

    @staticmethod
    def footprint(nx, ny, storage="f32", **prm):
        p = capi.make_params(nx, ny, storage=storage, **prm)
        return int(lib().lbm_pool_footprint(ctypes.byref(p)))

    def admit(self, mask, rhoA0, rhoB0, nsteps, noalloc=False, **prm):
        """Returns the slot id, or None when no slot or budget is free (LBM_EAGAIN).
        noalloc=True uses lbm_pool_admit_noalloc (no device allocation)."""
        mask = np.ascontiguousarray(mask, np.uint8)
        ny, nx = mask.shape
        p = capi.make_params(nx, ny, storage=self.storage, **prm)
        rA = _host(rhoA0, np.float64, mask.shape)
        rB = _host(rhoB0, np.float64, mask.shape)
        slot = ctypes.c_int32()
        fn = lib().lbm_pool_admit_noalloc if noalloc else lib().lbm_pool_admit
        code = fn(self._h, ctypes.byref(p), _p(mask), _p(rA), _p(rB), int(nsteps), ctypes.byref(slot))
        if code == capi.LBM_EAGAIN:
            return None
        check(code)
        self.shapes[slot.value] = (ny, nx)
        self._state_bytes[slot.value] = int(lib().lbm_params_state_bytes(ctypes.byref(p)))
        return slot.value

    def advance(self, chunk):
        check(lib().lbm_pool_advance(self._h, int(chunk)))

    def poll(self, max_n=256):
        out = (ctypes.c_int32 * max_n)()
        n = ctypes.c_int32()
        check(lib().lbm_pool_poll(self._h, out, int(max_n), ctypes.byref(n)))
        return [out[i] for i in range(n.value)]

    def fields(self, slot, raise_on_flags=True):
        ny, nx = self.shapes[slot]
        a = [np.zeros((ny, nx)) for _ in range(4)]
        _checked(lib().lbm_pool_fields(self._h, int(slot), *[_p(x) for x in a]), raise_on_flags=raise_on_flags)
        return tuple(a)

    def status(self, slot) -> int:
        """LBM_OK, or LBM_ENUMERIC once poll() has reported the slot broken (no device wait)."""
        code = int(lib().lbm_pool_status(self._h, int(slot)))
        if code not in (capi.LBM_OK, capi.LBM_ENUMERIC):
            check(code)
        return code

    def diag(self, slot, raise_on_flags=True):
        d = capi.LbmDiag()
        _checked(lib().lbm_pool_diag(self._h, int(slot), ctypes.byref(d)), raise_on_flags=raise_on_flags)
        return _diag_dict(d)

    def get_state(self, slot):
        buf = np.zeros(self._state_bytes[slot], np.uint8)
        check(lib().lbm_pool_get_state(self._h, int(slot), _p(buf)))
        return buf

    def set_state(self, slot, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        assert buf.size == self._state_bytes[slot]
        check(lib().lbm_pool_set_state(self._h, int(slot), _p(buf)))

    def release(self, slot):
        check(lib().lbm_pool_release(self._h, int(slot)))
        self.shapes.pop(slot, None)
        self._state_bytes.pop(slot, None)

    def progress(self):
        """(launches enqueued, launches completed on the device)."""
        a = ctypes.c_int64()
        b = ctypes.c_int64()
        check(lib().lbm_pool_progress(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def stats(self):
        a = ctypes.c_int32()
        b = ctypes.c_size_t()
        check(lib().lbm_pool_stats(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lbm_pool_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
