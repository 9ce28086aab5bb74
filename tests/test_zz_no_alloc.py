"""lbm_get_state_noalloc against lbm_get_state through the C ABI (needs an
MI355X; collected last): bitwise the same state and side state on two calls in a row, the
second on a smaller grid; no allocation through the grid's allocator during
the call; rows wider than the staging array rejected."""
import ctypes as ct
import os

import numpy as np
import pytest

from gpu_util import say
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu

ALLOC = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class CountingAllocator:
    """Device memory from hipMalloc / hipFree of the HIP runtime the library
    itself is bound to (called through ctypes), with call counts."""

    def __init__(self):
        lbm.load()
        self.hip = ct.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
        self.hip.hipMalloc.argtypes = [ct.POINTER(ct.c_void_p), ct.c_size_t]
        self.hip.hipFree.argtypes = [ct.c_void_p]
        self.allocs = 0
        self.frees = 0
        self._a = ALLOC(self._alloc)
        self._f = FREE(self._free)
        self.desc = lbm.lbm_allocator(ct.cast(self._a, ct.c_void_p), ct.cast(self._f, ct.c_void_p), None)

    def _alloc(self, nbytes, ctx):
        self.allocs += 1
        p = ct.c_void_p()
        return p.value if self.hip.hipMalloc(ct.byref(p), nbytes) == 0 else None

    def _free(self, ptr, ctx):
        self.frees += 1
        self.hip.hipFree(ptr)


def _export_both(g, alloc):
    n0 = (alloc.allocs, alloc.frees)
    Pn, sn = g.get_state_noalloc()
    n1 = (alloc.allocs, alloc.frees)
    Pa, sa = g.get_state()
    n2 = (alloc.allocs, alloc.frees)
    assert n1 == n0, "the allocation-free export allocated"
    assert n2[0] > n1[0], "the allocating export is expected to allocate its staging buffer"
    return (Pn, sn), (Pa, sa)


def test_noalloc_state_export_matches_twice():
    alloc = CountingAllocator()
    # first call: a 256 x 4096 D2Q21 annulus in FP32 (inner radius 640, cells
    # of aspect 0.98 to 1.37) whose FP64 state (176 MB) passes through the
    # 8 MiB staging array in 22 chunks of 12 rows (the last one 4 rows); moving
    # inner wall, so the side state is non-trivial
    big = G.circular_couette(21, 256, 4096, 640.0, u_inner=0.05, tau=0.8)
    rows_per_chunk = (8 << 20) // (21 * 4096 * 8)
    say("noalloc export: 256 x 4096 FP32, rows per chunk", rows_per_chunk)
    assert rows_per_chunk == 12 and 256 % rows_per_chunk == 4
    g = lbm.Grid(big, precision=lbm.LBM_FP32, alloc=alloc.desc)
    g.init()
    g.step(10)
    (Pn, sn), (Pa, sa) = _export_both(g, alloc)
    assert np.isfinite(Pa).all() and (sa != 0).any()
    assert np.array_equal(Pn, Pa) and np.array_equal(sn, sa)
    g.close()
    # second call, smaller input: a 12 x 100 FP64 annulus, both walls moving
    small = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    g = lbm.Grid(small, precision=lbm.LBM_FP64, alloc=alloc.desc)
    g.init()
    g.step(7)
    (Pn, sn), (Pa, sa) = _export_both(g, alloc)
    say("noalloc export: 12 x 100 FP64 equal", np.array_equal(Pn, Pa), np.array_equal(sn, sa))
    assert np.isfinite(Pa).all()
    assert np.array_equal(Pn, Pa) and np.array_equal(sn, sa)
    g.close()


def test_noalloc_state_export_rejects_rows_wider_than_staging():
    # q * n2 * 8 = 21 * 50000 * 8 bytes per row > 8 MiB
    case = G.planar_couette(21, G.faces_uniform(3), n2=50000, u_wall=0.05, tau=0.8)
    g = lbm.Grid(case, precision=lbm.LBM_FP32)
    g.init()
    with pytest.raises(lbm.LbmError) as e:
        g.get_state_noalloc()
    assert e.value.code == lbm.LBM_EINVAL
    assert "staging" in str(e.value)
    # the side state alone still fits
    side = np.zeros((2, 2, 3, 50000))
    rc = lbm.load().lbm_get_state_noalloc(g.h, None, side.ctypes.data_as(ct.POINTER(ct.c_double)))
    assert rc == lbm.LBM_OK
    g.close()
