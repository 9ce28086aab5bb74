"""The C-ABI library loads without a GPU and exports every declared symbol."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2301_01868_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2301_01868_amd import build
        build.build()
    return lbm.load()


def test_exports_every_declared_symbol(lib):
    from paper_2301_01868_amd import lbm3d
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            hdr = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char|void \*)\s*\*?\s*(lbm\w*_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 30 and "lbm3d_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert names <= set(lbm.EXPORTED) | set(lbm3d.EXPORTED) | {"lbm_lattice"}


def test_library_3d_lattice_agrees_with_oracle(lib):
    from paper_2301_01868_amd import lbm3d
    from oracle.oracle3d import lattice3
    c, w, T0 = lbm3d.lbm3d_lattice()
    oc, ow, oT0 = lattice3()
    assert np.array_equal(c, oc) and np.array_equal(w, ow) and T0 == oT0


def test_library_lattice_tables_agree_with_oracle(lib):
    for q in (9, 21):
        c, w, T0 = lbm.lbm_lattice(q)
        oc, ow, oT0, *_ = oracle.lattice(q)
        assert (c == oc).all() and np.array_equal(w, ow) and T0 == oT0


def test_bad_arguments_are_rejected(lib):
    from paper_2301_01868_amd import grids as G
    case = G.planar_couette(21, G.faces_uniform(8), n2=4)
    with pytest.raises(lbm.LbmError) as e:
        lbm.Grid(case.replace(tau=0.5))
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError):
        lbm.Grid(case.replace(halo=2))
    with pytest.raises(lbm.LbmError):
        lbm.Grid(G.planar_couette(21, G.faces_uniform(2), n2=4))


def _desc_case(**kw):
    """A Case whose coordinate arrays are placeholders: every case built here
    is rejected by the argument checks before the library reads them."""
    from paper_2301_01868_amd import grids as G
    return G.planar_couette(21, G.faces_uniform(8), n2=4).replace(**kw)


@pytest.mark.parametrize("kw,msg", [
    (dict(n1=0), "n1 and n2 must be positive"),
    (dict(n2=0), "n1 and n2 must be positive"),
    (dict(q=15), "q must be 9 or 21"),
    # 7 FP64 D2Q21 rows of 4,000,000 cells: 4.7 GB, past the 32-bit offsets of a row window
    (dict(n1=8, n2=4_000_000), "rows too long"),
    (dict(n1=1 << 16, n2=1 << 15), "grid too large"),
    (dict(n1=70000, n2=4), "n1 + 2 halo must not exceed 65535"),
])
def test_create_rejects_shapes(lib, kw, msg):
    with pytest.raises(lbm.LbmError) as e:
        lbm.Grid(_desc_case(**kw))
    assert e.value.code == lbm.LBM_EINVAL
    assert msg in str(e.value)


def test_create_rejects_modes(lib):
    case = _desc_case()
    for kw in (dict(precision=7), dict(iterations=17), dict(iterations=-1), dict(geometry=3), dict(geometry=-1)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.Grid(case, **kw)
        assert e.value.code == lbm.LBM_EINVAL, kw
    # a periodic q1 side must be paired with a periodic one
    with pytest.raises(lbm.LbmError) as e:
        lbm.Grid(case.replace(bc_lo="periodic", bc_hi="noslip"))
    assert e.value.code == lbm.LBM_EINVAL


def test_null_arguments_are_rejected(lib):
    import ctypes as ct
    h = ct.c_void_p()
    assert lib.lbm_grid_create(None, ct.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_batch_create(None, 1, ct.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_batch_create_ex(None, 1, 0, ct.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_batch_update(None, None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_grid_set_stream(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_init(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_step(None, ct.c_int64(1)) == lbm.LBM_EINVAL
    assert lib.lbm_set_occupancy(None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_batch_autotune(None, 10) == lbm.LBM_EINVAL
    w, c = ct.c_int32(), ct.c_int32()
    assert lib.lbm_batch_group_launch(None, 0, ct.byref(w), ct.byref(c)) == lbm.LBM_EINVAL
    assert lib.lbm_map_planar(3, 2, 2, None, 1.0, None, None) == lbm.LBM_EINVAL


def test_header_is_c_and_links_from_c(lib, tmp_path):
    """include/lbm.h compiles as strict C99 and the library links from C; the
    host-only lattice call runs without a GPU."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "abi.c"
    src.write_text(
        '#include "lbm.h"\n#include <stdio.h>\n'
        "int main(void) {\n"
        "    int32_t cx[21], cy[21]; double w[21], T0 = 0.0;\n"
        "    lbm_grid_desc d = {0}; lbm_resid r = {0}; lbm_grid_info info = {0};\n"
        "    (void)d; (void)r; (void)info;\n"
        "    if (lbm_lattice(21, cx, cy, w, &T0) != LBM_OK) return 1;\n"
        "    if (lbm_lattice(15, cx, cy, w, &T0) != LBM_EINVAL) return 2;\n"
        "    double f[4] = {0.0, 1.0, 2.0, 3.0}, x[11 * 10], y[11 * 10];\n"
        "    if (lbm_map_planar(3, 2, 4, f, 0.5, x, y) != LBM_OK) return 3;\n"
        "    if (lbm_map_planar(3, 2, 4, f, -1.0, x, y) != LBM_EINVAL) return 4;\n"
        '    printf("%.17g %d %d %.17g %.17g\\n", T0, cx[17], cy[18], x[0], y[10 * 10 - 1]);\n'
        "    return 0;\n}\n")
    exe = tmp_path / "abi"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                           os.path.join(ROOT, "include"), "-o", str(exe), str(src), lbm.LIB_PATH,
                           "-Wl,-rpath," + os.path.dirname(lbm.LIB_PATH)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert float(out[0]) == 2.0 / 3.0 and out[1:3] == ["3", "3"]
    # first ghost row of a 3-cell channel with halo 4 (rows -3..6 at x = 1/2 + integer); y of the last column
    assert float(out[3]) == -3.5 and float(out[4]) == (5 + 0.5) * 0.5


def test_unknown_offset_base_is_rejected(lib):
    with pytest.raises(lbm.LbmError) as e:
        lbm.Grid(_desc_case(), precision=lbm.LBM_FP32, offset_base=3)
    assert e.value.code == lbm.LBM_EINVAL
    assert "offset base" in str(e.value)


def test_noalloc_state_export_rejects_null_grid(lib):
    P = np.zeros(4)
    rc = lib.lbm_get_state_noalloc(None, P.ctypes.data_as(lbm.ct.POINTER(lbm.ct.c_double)), None)
    assert rc == lbm.LBM_EINVAL
