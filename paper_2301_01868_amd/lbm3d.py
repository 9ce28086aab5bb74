"""Thin ctypes binding of the 3D C ABI in include/lbm3d.h (argument
marshalling only; the library is the same liblbm.so as ``lbm``)."""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import lbm as _lbm

Q3 = 39
LbmError = _lbm.LbmError
BC = _lbm.BC


class lbm3d_grid_desc(ct.Structure):
    _fields_ = [("n1", ct.c_int32), ("n2", ct.c_int32), ("n3", ct.c_int32), ("halo", ct.c_int32),
                ("x", ct.POINTER(ct.c_double)), ("y", ct.POINTER(ct.c_double)), ("z", ct.POINTER(ct.c_double)),
                ("bc_lo", ct.c_int32), ("bc_hi", ct.c_int32), ("ut_lo", ct.c_double * 2), ("ut_hi", ct.c_double * 2),
                ("tau", ct.c_double), ("accel", ct.c_double * 3), ("rho0", ct.c_double), ("stream", ct.c_void_p)]


EXPORTED = ["lbm3d_lattice", "lbm3d_grid_create", "lbm3d_grid_destroy", "lbm3d_last_error", "lbm3d_init",
            "lbm3d_step", "lbm3d_moments", "lbm3d_get_state", "lbm3d_set_state", "lbm3d_stream_map",
            "lbm3d_geometry", "lbm3d_synchronize"]
_typed = False


def load():
    global _typed
    L = _lbm.load()
    if not _typed:
        D = ct.POINTER(ct.c_double)
        I32 = ct.POINTER(ct.c_int32)
        vp = ct.c_void_p
        L.lbm3d_lattice.argtypes = [I32, D, D]
        L.lbm3d_grid_create.argtypes = [ct.POINTER(lbm3d_grid_desc), ct.POINTER(vp)]
        L.lbm3d_grid_destroy.argtypes = [vp]
        L.lbm3d_grid_destroy.restype = None
        L.lbm3d_last_error.argtypes = [vp]
        L.lbm3d_last_error.restype = ct.c_char_p
        L.lbm3d_init.argtypes = [vp, D]
        L.lbm3d_step.argtypes = [vp, ct.c_int64]
        L.lbm3d_moments.argtypes = [vp, D, D, D]
        L.lbm3d_get_state.argtypes = [vp, D, D]
        L.lbm3d_set_state.argtypes = [vp, D, D]
        L.lbm3d_stream_map.argtypes = [vp, I32, I32, I32]
        L.lbm3d_geometry.argtypes = [vp, D]
        L.lbm3d_synchronize.argtypes = [vp]
        _typed = True
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def _chk(rc, h=None):
    if rc != 0:
        raise LbmError(rc, load().lbm3d_last_error(h).decode(errors="replace"))


def lbm3d_lattice():
    c = np.zeros((Q3, 3), dtype=np.int32)
    w = np.zeros(Q3)
    T0 = ct.c_double()
    _chk(load().lbm3d_lattice(c.ctypes.data_as(ct.POINTER(ct.c_int32)), _dp(w), ct.byref(T0)))
    return c, w, T0.value


class Grid3:
    """A 3D grid from a grids3d.Case3 (mapping + boundary + parameters)."""

    def __init__(self, case, stream=None):
        L = load()
        self.case = case
        self.n1, self.n2, self.n3 = case.n1, case.n2, case.n3
        self.ncell = case.ncell
        X = np.ascontiguousarray(case.X, dtype=np.float64)
        Y = np.ascontiguousarray(case.Y, dtype=np.float64)
        Z = np.ascontiguousarray(case.Z, dtype=np.float64)
        d = lbm3d_grid_desc()
        d.n1, d.n2, d.n3, d.halo = case.n1, case.n2, case.n3, case.halo
        d.x, d.y, d.z = _dp(X), _dp(Y), _dp(Z)
        d.bc_lo, d.bc_hi = BC[case.bc_lo], BC[case.bc_hi]
        if case.periodic1:
            d.bc_lo = d.bc_hi = 0
        d.ut_lo[0], d.ut_lo[1] = float(case.ut_lo[0]), float(case.ut_lo[1])
        d.ut_hi[0], d.ut_hi[1] = float(case.ut_hi[0]), float(case.ut_hi[1])
        d.tau = float(case.tau)
        for e in range(3):
            d.accel[e] = float(case.accel[e])
        d.rho0 = float(case.rho0)
        d.stream = stream
        h = ct.c_void_p()
        _chk(L.lbm3d_grid_create(ct.byref(d), ct.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().lbm3d_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, u0=None):
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).reshape(self.ncell, 3)
        _chk(load().lbm3d_init(self.h, _dp(u0)), self.h)

    def step(self, n=1):
        _chk(load().lbm3d_step(self.h, int(n)), self.h)

    def moments(self):
        m = np.zeros(self.ncell)
        U = np.zeros((self.ncell, 3))
        Ut = np.zeros((self.ncell, 3))
        _chk(load().lbm3d_moments(self.h, _dp(m), _dp(U), _dp(Ut)), self.h)
        return m, U, Ut

    def get_state(self):
        P = np.zeros((Q3, self.ncell))
        side = np.zeros((2, 3, 3, self.n2, self.n3))
        _chk(load().lbm3d_get_state(self.h, _dp(P), _dp(side)), self.h)
        return P, side

    def set_state(self, P=None, side=None):
        P = None if P is None else np.ascontiguousarray(P, dtype=np.float64)
        side = None if side is None else np.ascontiguousarray(side, dtype=np.float64)
        _chk(load().lbm3d_set_state(self.h, _dp(P), _dp(side)), self.h)

    def stream_map(self):
        n = self.ncell * Q3
        sc = np.zeros(n, np.int32)
        sd = np.zeros(n, np.int32)
        wl = np.zeros(n, np.int32)
        I32 = ct.POINTER(ct.c_int32)
        _chk(load().lbm3d_stream_map(self.h, sc.ctypes.data_as(I32), sd.ctypes.data_as(I32), wl.ctypes.data_as(I32)),
             self.h)
        return sc.reshape(-1, Q3), sd.reshape(-1, Q3), wl.reshape(-1, Q3)

    def geometry(self):
        out = np.zeros((self.ncell, 7 + 3 * Q3))
        _chk(load().lbm3d_geometry(self.h, _dp(out)), self.h)
        return out

    def synchronize(self):
        _chk(load().lbm3d_synchronize(self.h), self.h)
