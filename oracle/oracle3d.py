"""ctypes wrapper of the plain FP64 3D C oracle (``lbm_oracle3d.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Layouts follow the C
file: interior cells (i, j, k) with q3 fastest, populations cell-major
``P[cell, alpha]``; the mapping is given on the halo-extended range.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle3d.c")
_LIB = os.path.join(_HERE, "liblbm_oracle3d.so")
_lib = None
Q = 39
BC = {"periodic": 0, "noslip": 1, "moving": 2}


def build(force: bool = True) -> str:
    """Compile the 3D oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    L = ct.CDLL(_LIB)
    D = ct.POINTER(ct.c_double)
    I = ct.POINTER(ct.c_int)
    vp = ct.c_void_p
    L.o3_create.restype = vp
    L.o3_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, D, D, D, ct.c_int, ct.c_int, ct.c_int, D, D,
                            ct.c_double, D]
    L.o3_destroy.argtypes = [vp]
    L.o3_set_iterations.argtypes = [vp, ct.c_int]
    L.o3_init.argtypes = [vp, ct.c_double, D]
    L.o3_step.argtypes = [vp, ct.c_long, ct.c_int]
    L.o3_get_step.restype = ct.c_long
    L.o3_get_step.argtypes = [vp]
    L.o3_get_state.argtypes = [vp, D]
    L.o3_set_state.argtypes = [vp, D]
    L.o3_get_side.argtypes = [vp, D, D]
    L.o3_set_side.argtypes = [vp, D, D]
    L.o3_moments.argtypes = [vp, D, D, D]
    L.o3_step_cells.argtypes = [vp, ct.c_int, I, D]
    L.o3_geometry.argtypes = [vp, D]
    L.o3_stream_map.argtypes = [vp, I, I, I]
    L.o3_lattice.argtypes = [I, D, D]
    L.o3_feq.argtypes = [ct.c_double, D, D, D, D]
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ip(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_int))


def lattice3():
    """Velocity vectors c[39, 3], weights w[39], T0."""
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    T0 = ct.c_double()
    _load().o3_lattice(_ip(c), _dp(w), ct.byref(T0))
    return c, w, T0.value


def feq3(rho, U, Ut, G6):
    """Literal equilibrium (Eq. equilibrium, i, j, k over 1..3) for one cell;
    G6 = (g11, g12, g13, g22, g23, g33)."""
    out = np.zeros(Q)
    U = np.ascontiguousarray(U, dtype=np.float64)
    Ut = np.ascontiguousarray(Ut, dtype=np.float64)
    G6 = np.ascontiguousarray(G6, dtype=np.float64)
    _load().o3_feq(float(rho), _dp(U), _dp(Ut), _dp(G6), _dp(out))
    return out


class Oracle3D:
    """One 3D curvilinear grid stepped by the FP64 oracle."""

    def __init__(self, case):
        L = _load()
        self.case = case
        self.n1, self.n2, self.n3, self.h = case.n1, case.n2, case.n3, case.halo
        self.ncell = self.n1 * self.n2 * self.n3
        self.X = np.ascontiguousarray(case.X, dtype=np.float64)
        self.Y = np.ascontiguousarray(case.Y, dtype=np.float64)
        self.Z = np.ascontiguousarray(case.Z, dtype=np.float64)
        ut_lo = np.ascontiguousarray(case.ut_lo, dtype=np.float64)
        ut_hi = np.ascontiguousarray(case.ut_hi, dtype=np.float64)
        a = np.ascontiguousarray(case.accel, dtype=np.float64)
        self._h = L.o3_create(case.n1, case.n2, case.n3, case.halo, _dp(self.X), _dp(self.Y), _dp(self.Z),
                              int(case.periodic1), BC[case.bc_lo], BC[case.bc_hi], _dp(ut_lo), _dp(ut_hi),
                              float(case.tau), _dp(a))
        if not self._h:
            raise ValueError("3D oracle rejected the grid description")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().o3_destroy(self._h)
            self._h = None

    def set_iterations(self, k):
        _load().o3_set_iterations(self._h, int(k))

    def init(self, rho0=1.0, u0=None):
        if u0 is None:
            _load().o3_init(self._h, float(rho0), None)
        else:
            u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(self.ncell, 3)
            _load().o3_init(self._h, float(rho0), _dp(u0))

    def step(self, n=1, threads=0):
        _load().o3_step(self._h, int(n), int(threads))

    @property
    def t(self):
        return int(_load().o3_get_step(self._h))

    def get_state(self):
        P = np.zeros((self.ncell, Q))
        _load().o3_get_state(self._h, _dp(P))
        return P

    def set_state(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(self.ncell, Q)
        _load().o3_set_state(self._h, _dp(P))

    def get_side(self):
        m = np.zeros(self.ncell)
        u = np.zeros((self.ncell, 3))
        _load().o3_get_side(self._h, _dp(m), _dp(u))
        return m, u

    def set_side(self, m, u):
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(self.ncell)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.ncell, 3)
        _load().o3_set_side(self._h, _dp(m), _dp(u))

    def moments(self):
        """(m, U, Ut) the next step would see; U and Ut contravariant [cell][3]."""
        m = np.zeros(self.ncell)
        U = np.zeros((self.ncell, 3))
        Ut = np.zeros((self.ncell, 3))
        _load().o3_moments(self._h, _dp(m), _dp(U), _dp(Ut))
        return m, U, Ut

    def step_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        out = np.zeros((len(cells), Q))
        _load().o3_step_cells(self._h, len(cells), _ip(cells), _dp(out))
        return out

    def geometry(self):
        W = 1 + 6 + 9 + 3 * Q
        out = np.zeros((self.ncell, W))
        _load().o3_geometry(self._h, _dp(out))
        return {"J": out[:, 0].copy(), "G": out[:, 1:7].copy(), "g": out[:, 7:16].reshape(-1, 3, 3).copy(),
                "Aplus": out[:, 16:].reshape(-1, Q, 3).copy()}

    def stream_map(self):
        n = self.ncell * Q
        sc = np.zeros(n, dtype=np.int32)
        sd = np.zeros(n, dtype=np.int32)
        wl = np.zeros(n, dtype=np.int32)
        _load().o3_stream_map(self._h, _ip(sc), _ip(sd), _ip(wl))
        return sc.reshape(self.ncell, Q), sd.reshape(self.ncell, Q), wl.reshape(self.ncell, Q)

    def physical_velocity(self, Ut=None):
        """u = Ut^i g_i per cell."""
        if Ut is None:
            _, _, Ut = self.moments()
        g = self.geometry()["g"]
        return np.einsum("ci,cid->cd", Ut, g)
