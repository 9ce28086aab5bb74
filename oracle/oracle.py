"""ctypes wrapper of the plain FP64 C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Layouts follow the C
file: interior cells row-major with q2 fastest, populations cell-major
``P[cell, alpha]``; the mapping is given on the halo-extended range.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

BC = {"periodic": 0, "noslip": 1, "moving": 2}


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracles (2D and 3D) with gcc (-O2, no FP contraction, OpenMP)."""
    from . import oracle3d
    oracle3d.build(force)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
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
    I32 = ct.POINTER(ct.c_int32)
    L.orc_create.restype = ct.c_void_p
    L.orc_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, D, D, ct.c_int, ct.c_int, ct.c_int,
                             ct.c_double, ct.c_double, ct.c_double, ct.c_double, ct.c_double]
    L.orc_destroy.argtypes = [ct.c_void_p]
    L.orc_set_volume.argtypes = [ct.c_void_p, D]
    L.orc_init.argtypes = [ct.c_void_p, ct.c_double, D]
    L.orc_step.argtypes = [ct.c_void_p, ct.c_long, ct.c_int]
    L.orc_get_step.restype = ct.c_long
    L.orc_get_step.argtypes = [ct.c_void_p]
    L.orc_get_state.argtypes = [ct.c_void_p, D]
    L.orc_set_state.argtypes = [ct.c_void_p, D]
    L.orc_get_side.argtypes = [ct.c_void_p, D, D, D]
    L.orc_set_side.argtypes = [ct.c_void_p, D, D]
    L.orc_moments.argtypes = [ct.c_void_p, D, D, D, ct.c_int]
    L.orc_step_cells.argtypes = [ct.c_void_p, ct.c_int, I, D]
    L.orc_cell_detail.argtypes = [ct.c_void_p, ct.c_int, D]
    L.orc_geometry.argtypes = [ct.c_void_p, D]
    L.orc_stream_map.argtypes = [ct.c_void_p, I32, I32, I32]
    L.orc_lattice.argtypes = [ct.c_int, I, I, D, D, I, I]
    L.orc_feq.argtypes = [ct.c_int, ct.c_double, D, D, D, D]
    L.orc_max_threads.restype = ct.c_int
    L.orc_set_iterations.argtypes = [ct.c_void_p, ct.c_int]
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def lattice(q: int):
    """Velocity vectors, weights, T0, bounce-back and specular maps."""
    L = _load()
    cx = (ct.c_int * q)()
    cy = (ct.c_int * q)()
    w = np.zeros(q)
    T0 = ct.c_double()
    bb = (ct.c_int * q)()
    sp = (ct.c_int * q)()
    L.orc_lattice(q, cx, cy, _dp(w), ct.byref(T0), bb, sp)
    c = np.stack([np.array(cx[:]), np.array(cy[:])], axis=1)
    return c, w, T0.value, np.array(bb[:]), np.array(sp[:])


def feq(q: int, rho: float, U, Ut, G3) -> np.ndarray:
    """Literal equilibrium (Eq. equilibrium) for one cell; G3 = (g11, g12, g22)."""
    L = _load()
    U = np.ascontiguousarray(U, dtype=np.float64)
    Ut = np.ascontiguousarray(Ut, dtype=np.float64)
    G3 = np.ascontiguousarray(G3, dtype=np.float64)
    out = np.zeros(q)
    L.orc_feq(q, float(rho), _dp(U), _dp(Ut), _dp(G3), _dp(out))
    return out


class OracleGrid:
    """One curvilinear grid stepped by the FP64 oracle."""

    def __init__(self, case):
        L = _load()
        self.case = case
        self.q, self.n1, self.n2, self.h = case.q, case.n1, case.n2, case.halo
        self.X = np.ascontiguousarray(case.X, dtype=np.float64)
        self.Y = np.ascontiguousarray(case.Y, dtype=np.float64)
        assert self.X.shape == (self.n1 + 2 * self.h, self.n2 + 2 * self.h)
        self._h = L.orc_create(case.q, case.n1, case.n2, case.halo, _dp(self.X), _dp(self.Y),
                               int(case.periodic1), BC[case.bc_lo], BC[case.bc_hi], float(case.ut_lo),
                               float(case.ut_hi), float(case.tau), float(case.accel[0]), float(case.accel[1]))
        if not self._h:
            raise ValueError("oracle rejected the grid description")
        self.ncell = self.n1 * self.n2

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_destroy(self._h)
            self._h = None

    # -- state ------------------------------------------------------------
    def init(self, rho0=1.0, u0=None):
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(self.ncell, 2)
            _load().orc_init(self._h, rho0, _dp(u0))
        else:
            _load().orc_init(self._h, rho0, None)

    def set_volume(self, J=None):
        if J is None:
            _load().orc_set_volume(self._h, None)
        else:
            J = np.ascontiguousarray(J, dtype=np.float64).reshape(self.ncell)
            _load().orc_set_volume(self._h, _dp(J))

    def set_iterations(self, k):
        """0: lagged force (the paper's choice); k > 0: k fixed-point passes."""
        _load().orc_set_iterations(self._h, int(k))

    def step(self, n=1, threads=0):
        _load().orc_step(self._h, int(n), int(threads))

    @property
    def t(self):
        return int(_load().orc_get_step(self._h))

    def get_state(self):
        P = np.zeros((self.ncell, self.q))
        _load().orc_get_state(self._h, _dp(P))
        return P

    def set_state(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(self.ncell, self.q)
        _load().orc_set_state(self._h, _dp(P))

    def get_side(self):
        m = np.zeros(self.ncell)
        u1 = np.zeros(self.ncell)
        u2 = np.zeros(self.ncell)
        _load().orc_get_side(self._h, _dp(m), _dp(u1), _dp(u2))
        return m, u1, u2

    def set_side(self, m, u2):
        m = np.ascontiguousarray(m, dtype=np.float64).reshape(self.ncell)
        u2 = np.ascontiguousarray(u2, dtype=np.float64).reshape(self.ncell)
        _load().orc_set_side(self._h, _dp(m), _dp(u2))

    # -- outputs ----------------------------------------------------------
    def moments(self, threads=0):
        """(m, U, Ut) of the next pre-collision state, U and Ut contravariant."""
        m = np.zeros(self.ncell)
        U = np.zeros((self.ncell, 2))
        Ut = np.zeros((self.ncell, 2))
        _load().orc_moments(self._h, _dp(m), _dp(U), _dp(Ut), int(threads))
        return m, U, Ut

    def step_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int32)
        out = np.zeros((len(cells), self.q))
        _load().orc_step_cells(self._h, len(cells), cells.ctypes.data_as(ct.POINTER(ct.c_int)), _dp(out))
        return out

    def cell_detail(self, cell):
        Q = self.q
        out = np.zeros(Q + 8 + Q + 4 + Q + Q)
        _load().orc_cell_detail(self._h, int(cell), _dp(out))
        o = 0
        d = {}
        d["N"] = out[o:o + Q]; o += Q
        d["m"], d["rho"] = out[o], out[o + 1]; o += 2
        d["U"] = out[o:o + 2]; o += 2
        d["F"] = out[o:o + 2]; o += 2
        d["Ut"] = out[o:o + 2]; o += 2
        d["feq"] = out[o:o + Q]; o += Q
        d["dPi"] = out[o:o + 4].reshape(2, 2); o += 4
        d["dN"] = out[o:o + Q]; o += Q
        d["Np"] = out[o:o + Q]; o += Q
        return d

    def geometry(self):
        """Per-cell J, G (3), g1, g2, Aplus[Q,2], Aminus[Q,2] as a dict."""
        Q = self.q
        W = 8 + 4 * Q
        out = np.zeros((self.ncell, W))
        _load().orc_geometry(self._h, _dp(out))
        return {
            "J": out[:, 0].copy(), "G": out[:, 1:4].copy(), "g1": out[:, 4:6].copy(), "g2": out[:, 6:8].copy(),
            "Aplus": out[:, 8:8 + 2 * Q].reshape(self.ncell, Q, 2).copy(),
            "Aminus": out[:, 8 + 2 * Q:8 + 4 * Q].reshape(self.ncell, Q, 2).copy(),
        }

    def stream_map(self):
        n = self.ncell * self.q
        sc = np.zeros(n, dtype=np.int32)
        sd = np.zeros(n, dtype=np.int32)
        wl = np.zeros(n, dtype=np.int32)
        I32 = ct.POINTER(ct.c_int32)
        _load().orc_stream_map(self._h, sc.ctypes.data_as(I32), sd.ctypes.data_as(I32), wl.ctypes.data_as(I32))
        return sc.reshape(self.ncell, self.q), sd.reshape(self.ncell, self.q), wl.reshape(self.ncell, self.q)

    # -- derived diagnostics (plain definitions, Sec. 3 text) ----------------
    def physical_velocity(self, Ut=None):
        """u = Utilde^i g_i(q) (Eq. result with the physical velocity)."""
        if Ut is None:
            _, _, Ut = self.moments()
        geo = self.geometry()
        return Ut[:, 0:1] * geo["g1"] + Ut[:, 1:2] * geo["g2"]
