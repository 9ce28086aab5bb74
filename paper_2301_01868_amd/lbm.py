"""Thin ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

Every function has the ABI's name and forwards to ``liblbm.so``; nothing here
computes any step of the method.  Loading fails loudly when the library has
not been built (``python -m paper_2301_01868_amd.build``).

PyTorch ships its own HIP runtime with the same soname (libamdhip64.so.7) as
the ROCm one the library links.  Whichever is loaded first serves both, but
torch's device initialisation fails on the ROCm one ("no ROCm-capable
device"), so ``load()`` imports torch (when it is installed) before it opens
the library: torch streams and torch memory then work with the library in
any order of use.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_PERIODIC, LBM_NOSLIP, LBM_MOVING = 0, 1, 2
LBM_FP64, LBM_FP32, LBM_FP16 = 0, 1, 2
LBM_BASE_LOCAL_REST, LBM_BASE_W_RHO0, LBM_BASE_NONE = 0, 1, 2
LBM_GEOM_AUTO, LBM_GEOM_CELL, LBM_GEOM_CELL_TABLE = 0, 1, 2
LBM_BATCH_FUSE_LATTICES = 1
BC = {"periodic": LBM_PERIODIC, "noslip": LBM_NOSLIP, "moving": LBM_MOVING}

EXPORTED = ["lbm_lattice", "lbm_grid_create", "lbm_grid_destroy", "lbm_last_error", "lbm_grid_info_get",
            "lbm_set_volume", "lbm_get_volume", "lbm_init", "lbm_step", "lbm_moments", "lbm_residual", "lbm_noflow_adjust",
            "lbm_get_state", "lbm_set_state", "lbm_save", "lbm_load", "lbm_physical_velocity", "lbm_stream_map", "lbm_geometry", "lbm_synchronize",
            "lbm_stream", "lbm_batch_create", "lbm_batch_create_ex", "lbm_batch_step", "lbm_batch_destroy", "lbm_batch_residuals", "lbm_batch_info", "lbm_batch_step_group", "lbm_set_launch", "lbm_set_occupancy", "lbm_autotune",
            "lbm_copy_probe", "lbm_bandwidth_probe", "lbm_map_planar", "lbm_map_polar",
            "lbm_batch_autotune", "lbm_batch_group_launch", "lbm_get_state_noalloc", "lbm_grid_set_stream",
            "lbm_batch_update"]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm error %d: %s" % (code, msg))
        self.code = code


class lbm_allocator(ct.Structure):
    _fields_ = [("alloc", ct.c_void_p), ("free", ct.c_void_p), ("ctx", ct.c_void_p)]


class lbm_grid_desc(ct.Structure):
    _fields_ = [("q", ct.c_int32), ("n1", ct.c_int32), ("n2", ct.c_int32), ("halo", ct.c_int32),
                ("x", ct.POINTER(ct.c_double)), ("y", ct.POINTER(ct.c_double)),
                ("bc_lo", ct.c_int32), ("bc_hi", ct.c_int32), ("ut_lo", ct.c_double), ("ut_hi", ct.c_double),
                ("tau", ct.c_double), ("accel", ct.c_double * 2), ("rho0", ct.c_double),
                ("precision", ct.c_int32), ("offset_base", ct.c_int32), ("iterations", ct.c_int32),
                ("geometry", ct.c_int32), ("alloc", ct.POINTER(lbm_allocator)), ("stream", ct.c_void_p)]


class lbm_resid(ct.Structure):
    _fields_ = [("step", ct.c_int64), ("residual", ct.c_double), ("mass", ct.c_double),
                ("mass_rel_drift", ct.c_double), ("kinetic_energy", ct.c_double),
                ("angular_momentum", ct.c_double), ("bad_cells", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_grid_info(ct.Structure):
    _fields_ = [("q", ct.c_int32), ("n1", ct.c_int32), ("n2", ct.c_int32), ("pitch", ct.c_int32),
                ("precision", ct.c_int32), ("row_tables", ct.c_int32), ("step", ct.c_int64),
                ("bytes_per_update", ct.c_double), ("device_bytes", ct.c_size_t),
                ("waves_per_block", ct.c_int32), ("waves_per_cu_cap", ct.c_int32),
                ("table_kind", ct.c_int32), ("reserved", ct.c_int32)]


_lib = None


def load():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library not built: %s (run python -m paper_2301_01868_amd.build)" % LIB_PATH)
    try:
        import torch  # noqa: F401  (its HIP runtime first: see the module notes)
    except ImportError:
        pass
    L = ct.CDLL(LIB_PATH)
    D = ct.POINTER(ct.c_double)
    I32 = ct.POINTER(ct.c_int32)
    vp = ct.c_void_p
    L.lbm_lattice.argtypes = [ct.c_int32, I32, I32, D, D]
    L.lbm_grid_create.argtypes = [ct.POINTER(lbm_grid_desc), ct.POINTER(vp)]
    L.lbm_grid_destroy.argtypes = [vp]
    L.lbm_grid_destroy.restype = None
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ct.c_char_p
    L.lbm_grid_info_get.argtypes = [vp, ct.POINTER(lbm_grid_info)]
    L.lbm_set_volume.argtypes = [vp, D]
    L.lbm_init.argtypes = [vp, D]
    L.lbm_get_volume.argtypes = [vp, D]
    L.lbm_step.argtypes = [vp, ct.c_int64]
    L.lbm_moments.argtypes = [vp, D, D, D]
    L.lbm_residual.argtypes = [vp, ct.POINTER(lbm_resid)]
    L.lbm_noflow_adjust.argtypes = [vp, ct.c_double, ct.c_int64, ct.c_int32, ct.POINTER(ct.c_int64)]
    L.lbm_get_state.argtypes = [vp, D, D]
    L.lbm_set_state.argtypes = [vp, D, D]
    L.lbm_get_state_noalloc.argtypes = [vp, D, D]
    L.lbm_save.argtypes = [vp, vp, ct.POINTER(ct.c_size_t)]
    L.lbm_load.argtypes = [vp, vp, ct.c_size_t]
    L.lbm_physical_velocity.argtypes = [vp, D]
    L.lbm_stream_map.argtypes = [vp, I32, I32, I32]
    L.lbm_geometry.argtypes = [vp, D]
    L.lbm_synchronize.argtypes = [vp]
    L.lbm_stream.argtypes = [vp]
    L.lbm_stream.restype = vp
    L.lbm_grid_set_stream.argtypes = [vp, vp]
    L.lbm_batch_update.argtypes = [vp, ct.POINTER(vp), ct.c_int32]
    L.lbm_batch_create.argtypes = [ct.POINTER(vp), ct.c_int32, ct.POINTER(vp)]
    L.lbm_batch_create_ex.argtypes = [ct.POINTER(vp), ct.c_int32, ct.c_uint32, ct.POINTER(vp)]
    L.lbm_batch_step.argtypes = [vp, ct.c_int64]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_destroy.restype = None
    L.lbm_batch_residuals.argtypes = [vp, ct.POINTER(lbm_resid)]
    L.lbm_batch_info.argtypes = [vp, ct.c_int32, I32, I32, ct.POINTER(ct.c_int64)]
    L.lbm_batch_step_group.argtypes = [vp, ct.c_int32, ct.c_int64]
    L.lbm_set_launch.argtypes = [vp, ct.c_int32]
    L.lbm_set_occupancy.argtypes = [vp, ct.c_int32]
    L.lbm_autotune.argtypes = [vp, ct.c_int32]
    L.lbm_copy_probe.argtypes = [vp, vp, ct.c_size_t, vp]
    L.lbm_bandwidth_probe.argtypes = [vp, vp, ct.c_size_t, ct.c_int32, vp]
    L.lbm_batch_autotune.argtypes = [vp, ct.c_int32]
    L.lbm_batch_group_launch.argtypes = [vp, ct.c_int32, I32, I32]
    L.lbm_map_planar.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32, D, ct.c_double, D, D]
    L.lbm_map_polar.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32, D, ct.c_int32, D, D]
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ct.POINTER(ct.c_double))


def _chk(rc, handle=None):
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error(handle).decode(errors="replace"))
    return rc


# ---------------------------------------------------------------------------
# functions with the ABI's names
# ---------------------------------------------------------------------------
def lbm_lattice(q):
    cx = (ct.c_int32 * q)()
    cy = (ct.c_int32 * q)()
    w = np.zeros(q)
    T0 = ct.c_double()
    _chk(load().lbm_lattice(q, cx, cy, _dp(w), ct.byref(T0)))
    return np.stack([np.array(cx[:]), np.array(cy[:])], 1), w, T0.value


def lbm_map_planar(faces, n2, halo, d_per=1.0):
    """Halo-extended cell centres (X, Y) of a planar channel, shape (n1 + 2 halo, n2 + 2 halo)."""
    f = np.ascontiguousarray(faces, dtype=np.float64)
    n1 = len(f) - 1
    X = np.empty((n1 + 2 * halo, n2 + 2 * halo))
    Y = np.empty_like(X)
    _chk(load().lbm_map_planar(n1, n2, halo, _dp(f), d_per, _dp(X), _dp(Y)))
    return X, Y


def lbm_map_polar(r_faces, ntheta, halo, n2=None):
    """Halo-extended cell centres (X, Y) of an annulus on the half-spaced polar lattice."""
    f = np.ascontiguousarray(r_faces, dtype=np.float64)
    n1 = len(f) - 1
    n2 = ntheta if n2 is None else n2
    X = np.empty((n1 + 2 * halo, n2 + 2 * halo))
    Y = np.empty_like(X)
    _chk(load().lbm_map_polar(n1, n2, halo, _dp(f), ntheta, _dp(X), _dp(Y)))
    return X, Y


def lbm_grid_create(case, precision=LBM_FP64, offset_base=LBM_BASE_LOCAL_REST, iterations=0,
                    geometry=LBM_GEOM_AUTO, stream=None, alloc=None):
    """Create a grid from a grids.Case (mapping + boundary + parameters);
    `alloc` is an optional lbm_allocator the caller keeps alive for the
    grid's lifetime."""
    X = np.ascontiguousarray(case.X, dtype=np.float64)
    Y = np.ascontiguousarray(case.Y, dtype=np.float64)
    d = lbm_grid_desc()
    d.q, d.n1, d.n2, d.halo = case.q, case.n1, case.n2, case.halo
    d.x, d.y = _dp(X), _dp(Y)
    d.bc_lo, d.bc_hi = BC[case.bc_lo], BC[case.bc_hi]
    if case.periodic1:
        d.bc_lo = d.bc_hi = LBM_PERIODIC
    d.ut_lo, d.ut_hi = float(case.ut_lo), float(case.ut_hi)
    d.tau = float(case.tau)
    d.accel[0], d.accel[1] = float(case.accel[0]), float(case.accel[1])
    d.rho0 = float(case.rho0)
    d.precision, d.offset_base, d.iterations, d.geometry = precision, offset_base, iterations, geometry
    d.alloc = None if alloc is None else ct.pointer(alloc)
    d.stream = stream
    h = ct.c_void_p()
    _chk(load().lbm_grid_create(ct.byref(d), ct.byref(h)))
    return h


def lbm_grid_destroy(h):
    load().lbm_grid_destroy(h)


def lbm_grid_info_get(h):
    info = lbm_grid_info()
    _chk(load().lbm_grid_info_get(h, ct.byref(info)), h)
    return info


def lbm_set_volume(h, J=None):
    J = None if J is None else np.ascontiguousarray(J, dtype=np.float64)
    _chk(load().lbm_set_volume(h, _dp(J)), h)


def lbm_get_volume(h, ncell):
    J = np.zeros(ncell)
    _chk(load().lbm_get_volume(h, _dp(J)), h)
    return J


def lbm_init(h, u0=None):
    u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    _chk(load().lbm_init(h, _dp(u0)), h)


def lbm_step(h, n):
    _chk(load().lbm_step(h, int(n)), h)


def lbm_moments(h, ncell):
    m = np.zeros(ncell)
    U = np.zeros((ncell, 2))
    Ut = np.zeros((ncell, 2))
    _chk(load().lbm_moments(h, _dp(m), _dp(U), _dp(Ut)), h)
    return m, U, Ut


def lbm_residual(h, check=True):
    r = lbm_resid()
    rc = load().lbm_residual(h, ct.byref(r))
    if check:
        _chk(rc, h)
    return r


def lbm_noflow_adjust(h, tol=1e-12, max_steps=10 ** 7, check_every=1000):
    steps = ct.c_int64()
    _chk(load().lbm_noflow_adjust(h, float(tol), int(max_steps), int(check_every), ct.byref(steps)), h)
    return steps.value


def lbm_get_state(h, q, n1, n2, cmax):
    P = np.zeros((q, n1, n2))
    side = np.zeros((2, 2, cmax, n2))
    _chk(load().lbm_get_state(h, _dp(P), _dp(side)), h)
    return P, side


def lbm_get_state_noalloc(h, q, n1, n2, cmax, P=None, side=None):
    """As lbm_get_state, staged through the library's fixed device array (no
    allocation by the library); pass P [q][n1][n2] and side [2][2][cmax][n2]
    to reuse caller-owned host arrays."""
    P = np.zeros((q, n1, n2)) if P is None else P
    side = np.zeros((2, 2, cmax, n2)) if side is None else side
    assert P.dtype == np.float64 and P.flags.c_contiguous and P.size == q * n1 * n2
    assert side.dtype == np.float64 and side.flags.c_contiguous and side.size == 4 * cmax * n2
    _chk(load().lbm_get_state_noalloc(h, _dp(P), _dp(side)), h)
    return P, side


def lbm_set_state(h, P=None, side=None):
    P = None if P is None else np.ascontiguousarray(P, dtype=np.float64)
    side = None if side is None else np.ascontiguousarray(side, dtype=np.float64)
    _chk(load().lbm_set_state(h, _dp(P), _dp(side)), h)


def lbm_stream_map(h, ncell, q):
    sc = np.zeros((ncell, q), np.int32)
    sd = np.zeros((ncell, q), np.int32)
    wl = np.zeros((ncell, q), np.int32)
    I32 = ct.POINTER(ct.c_int32)
    _chk(load().lbm_stream_map(h, sc.ctypes.data_as(I32), sd.ctypes.data_as(I32), wl.ctypes.data_as(I32)), h)
    return sc, sd, wl


def lbm_geometry(h, ncell, q):
    out = np.zeros((ncell, 4 + 2 * q))
    _chk(load().lbm_geometry(h, _dp(out)), h)
    return out


def lbm_synchronize(h):
    _chk(load().lbm_synchronize(h), h)


def lbm_stream(h):
    return load().lbm_stream(h)


def lbm_grid_set_stream(h, stream):
    """Move the grid's later work to `stream` (a raw hipStream_t value, or
    None for a library-owned stream); queued work stays ordered before it."""
    _chk(load().lbm_grid_set_stream(h, stream), h)


def lbm_autotune(h, steps=20):
    rc = load().lbm_autotune(h, int(steps))
    if rc < 0:
        _chk(rc, h)
    return rc


def lbm_set_launch(h, waves_per_block):
    _chk(load().lbm_set_launch(h, int(waves_per_block)), h)


def lbm_set_occupancy(h, waves_per_cu):
    _chk(load().lbm_set_occupancy(h, int(waves_per_cu)), h)


def lbm_save(h):
    """Checkpoint blob of the grid's state (bytes)."""
    n = ct.c_size_t(0)
    _chk(load().lbm_save(h, None, ct.byref(n)), h)
    buf = ct.create_string_buffer(n.value)
    _chk(load().lbm_save(h, buf, ct.byref(n)), h)
    return buf.raw[:n.value]


def lbm_load(h, blob):
    buf = ct.create_string_buffer(bytes(blob), len(blob))
    _chk(load().lbm_load(h, buf, len(blob)), h)


def lbm_physical_velocity(h, ncell):
    u = np.zeros((ncell, 2))
    _chk(load().lbm_physical_velocity(h, _dp(u)), h)
    return u


def lbm_batch_create(handles):
    arr = (ct.c_void_p * len(handles))(*[h.value if isinstance(h, ct.c_void_p) else h for h in handles])
    b = ct.c_void_p()
    _chk(load().lbm_batch_create(arr, len(handles), ct.byref(b)))
    return b


def lbm_batch_create_ex(handles, flags=0):
    arr = (ct.c_void_p * len(handles))(*[h.value if isinstance(h, ct.c_void_p) else h for h in handles])
    b = ct.c_void_p()
    _chk(load().lbm_batch_create_ex(arr, len(handles), ct.c_uint32(flags), ct.byref(b)))
    return b


def lbm_batch_update(b, handles):
    """Make `handles` the batch's members in place (continuous batching)."""
    hs = [h.value if isinstance(h, ct.c_void_p) else h for h in handles]
    arr = (ct.c_void_p * max(1, len(hs)))(*hs)
    _chk(load().lbm_batch_update(b, arr, len(hs)))


def lbm_batch_step(b, n):
    _chk(load().lbm_batch_step(b, int(n)))


def lbm_batch_destroy(b):
    load().lbm_batch_destroy(b)


def lbm_batch_residuals(b, n, check=False):
    arr = (lbm_resid * n)()
    rc = load().lbm_batch_residuals(b, arr)
    if check:
        _chk(rc)
    elif rc not in (LBM_OK, LBM_EUNSTABLE):
        _chk(rc)
    return list(arr)


def lbm_batch_info(b, group):
    q = ct.c_int32()
    prec = ct.c_int32()
    cells = ct.c_int64()
    n = load().lbm_batch_info(b, int(group), ct.byref(q), ct.byref(prec), ct.byref(cells))
    if n < 0:
        _chk(n)
    return n, q.value, prec.value, cells.value


def lbm_batch_groups(b):
    n = load().lbm_batch_info(b, 0, None, None, None)
    if n < 0:
        _chk(n)
    return [lbm_batch_info(b, k)[1:] for k in range(n)]


def lbm_batch_autotune(b, steps=20):
    _chk(load().lbm_batch_autotune(b, steps))


def lbm_batch_group_launch(b, group):
    """(waves per workgroup, waves-per-CU cap) of a batch group's step launch."""
    w = ct.c_int32()
    c = ct.c_int32()
    _chk(load().lbm_batch_group_launch(b, group, ct.byref(w), ct.byref(c)))
    return w.value, c.value


def lbm_batch_step_group(b, group, n):
    _chk(load().lbm_batch_step_group(b, int(group), int(n)))


def lbm_bandwidth_probe(dst_ptr, src_ptr, nbytes, kind, stream=None):
    _chk(load().lbm_bandwidth_probe(ct.c_void_p(dst_ptr), ct.c_void_p(src_ptr), int(nbytes), int(kind), stream))


def lbm_copy_probe(dst_ptr, src_ptr, nbytes, stream=None):
    _chk(load().lbm_copy_probe(ct.c_void_p(dst_ptr), ct.c_void_p(src_ptr), int(nbytes), stream))


# ---------------------------------------------------------------------------
# a small object wrapper over the same calls
# ---------------------------------------------------------------------------
class Grid:
    def __init__(self, case, precision=LBM_FP64, offset_base=LBM_BASE_LOCAL_REST, iterations=0,
                 geometry=LBM_GEOM_AUTO, stream=None, alloc=None):
        self.case = case
        self.q, self.n1, self.n2 = case.q, case.n1, case.n2
        self.ncell = case.n1 * case.n2
        self.cmax = 1 if case.q == 9 else 3
        self._alloc = alloc        # kept alive with the grid
        self.h = lbm_grid_create(case, precision, offset_base, iterations, geometry, stream, alloc)

    def close(self):
        if getattr(self, "h", None):
            lbm_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        return lbm_grid_info_get(self.h)

    def set_volume(self, J=None):
        lbm_set_volume(self.h, J)

    def get_volume(self):
        return lbm_get_volume(self.h, self.ncell)

    def init(self, u0=None):
        lbm_init(self.h, u0)

    def step(self, n=1):
        lbm_step(self.h, n)

    def moments(self):
        return lbm_moments(self.h, self.ncell)

    def residual(self, check=True):
        return lbm_residual(self.h, check)

    def noflow_adjust(self, tol=1e-12, max_steps=10 ** 7, check_every=1000):
        return lbm_noflow_adjust(self.h, tol, max_steps, check_every)

    def save(self):
        return lbm_save(self.h)

    def load(self, blob):
        lbm_load(self.h, blob)

    def physical_velocity(self):
        return lbm_physical_velocity(self.h, self.ncell)

    def get_state(self):
        return lbm_get_state(self.h, self.q, self.n1, self.n2, self.cmax)

    def get_state_noalloc(self, P=None, side=None):
        return lbm_get_state_noalloc(self.h, self.q, self.n1, self.n2, self.cmax, P, side)

    def set_state(self, P=None, side=None):
        lbm_set_state(self.h, P, side)

    def stream_map(self):
        return lbm_stream_map(self.h, self.ncell, self.q)

    def geometry(self):
        return lbm_geometry(self.h, self.ncell, self.q)

    def synchronize(self):
        lbm_synchronize(self.h)

    def set_launch(self, wpb):
        lbm_set_launch(self.h, wpb)

    def set_occupancy(self, waves_per_cu):
        lbm_set_occupancy(self.h, waves_per_cu)

    def autotune(self, steps=20):
        return lbm_autotune(self.h, steps)

    @property
    def stream(self):
        return lbm_stream(self.h)

    def set_stream(self, stream):
        lbm_grid_set_stream(self.h, stream)
