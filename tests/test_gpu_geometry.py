"""Per-cell metric terms rebuilt in the step from the staged FP64 geometry
(LBM_GEOM_CELL, the default for mappings whose terms depend on q2), against
the FP64 oracle and against the stored per-cell tables (LBM_GEOM_CELL_TABLE)
(needs an MI355X).

The terms are those of Sec. 2: g^ij (Eq. covectors), the Christoffel sums
A+^i_a = g^i . [e_a(q + c_a) - e_a(q)] (Eqs. gamma, lattice) and, for offset
storage, the local rest state of the cell and of each pulled source."""
import numpy as np
import pytest

import oracle
from gpu_util import characteristic_speed, initial_velocity, norm_rel, one_step_sampled, pair, say, to_oracle_state
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu


def _cases():
    # q2-dependent mappings (per-cell terms by necessity): narrow and wide
    # (the wide rows take the kernel's unwrapped fast path), both lattices
    yield "box_wobble_q21_narrow", G.periodic_box(21, 9, 11, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    yield "box_wobble_q21_wide", G.periodic_box(21, 10, 150, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    yield "box_wobble_q9_wide", G.periodic_box(9, 12, 140, dx=1.0, dy=1.2, wobble=0.2, tau=0.8)
    # non-orthogonal and wall-bounded: the journal bearing (eccentric annulus),
    # inner wall sliding
    yield "eccentric_q21", G.eccentric_annulus(21, 16, 150, 16.0, 1.0, tau=1.0)
    yield "eccentric_q9", G.eccentric_annulus(9, 16, 150, 16.0, 2.0, tau=1.0)
    # row-invariant mappings forced onto the per-cell path: walls at rest,
    # moving walls (specular sources), a ragged last tile, a stretched channel
    yield "annulus_q21_moving", G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    yield "annulus_q21_wide", G.circular_couette(21, 9, 160, 25.0, u_inner=0.05, tau=0.8)
    yield "channel_q21_ragged", G.planar_couette(21, G.faces_linear(14, 0.35), n2=70, u_wall=0.04, moving="lo",
                                                  tau=0.7).replace(accel=(0.0, 2e-6))
    yield "couette_q9", G.workload_planar_couette_q9()
    # a channel of 3 rows between a resting and a moving wall: every D2Q21
    # source 3 rows out is the mirror of a row on the far side of the channel,
    # so the staged tile rows past both walls hold mirror rows
    yield "narrow_q21_moving", G.planar_couette(21, G.faces_uniform(3), n2=70, u_wall=0.03, tau=0.9)


CASES = list(_cases())


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_rebuilt_geometry_fp64_matches_oracle(name, case):
    g, o = pair(case, geometry=lbm.LBM_GEOM_CELL)
    assert g.info.table_kind == 2 and not g.info.row_tables
    g.step(300)
    o.step(300)
    P, _ = g.get_state()
    err = norm_rel(to_oracle_state(P), o.get_state())
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    say(name, "fp64 rebuilt geometry: state rel err %.2e" % err)
    assert err <= 1e-12
    assert np.abs(Ut - Uto).max() <= 1e-12 * max(np.abs(Uto).max(), 1e-3)


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_rebuilt_geometry_fp32_within_tolerance(name, case):
    """FP32 offsets from the local rest state, with the rest state of every
    pulled source evaluated in FP64 from the staged geometry: velocity within
    1e-5 of the characteristic speed of the FP64 oracle."""
    g, o = pair(case, precision=lbm.LBM_FP32, geometry=lbm.LBM_GEOM_CELL)
    g.step(300)
    o.step(300)
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    geo = o.geometry()
    u = Ut[:, :1] * geo["g1"] + Ut[:, 1:] * geo["g2"]
    uo = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    Uc = characteristic_speed(case, uo)
    err = np.abs(u - uo).max() / Uc
    say(name, "fp32 rebuilt geometry: velocity err / U %.2e" % err)
    assert err <= 1e-5
    assert norm_rel(m, mo) <= 1e-6


@pytest.mark.parametrize("base", [lbm.LBM_BASE_LOCAL_REST, lbm.LBM_BASE_W_RHO0], ids=["local_rest", "w_rho0"])
@pytest.mark.parametrize("prec", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16], ids=["fp64", "fp32", "fp16"])
def test_rebuilt_geometry_equals_stored_tables(prec, base):
    """On a larger wobbled box (several row tiles and column blocks, a ragged
    last block), rebuilt and stored per-cell terms give the same trajectory to
    the rounding of the compute type.  Offset storage with the w rho0 base
    reads the stored table even when rebuilt terms are asked for (its base
    differences need the table's FP64-rounded values): then both runs take
    the same kernel and agree bitwise."""
    case = G.periodic_box(21, 40, 300, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    u0 = initial_velocity(case)
    out = []
    rebuilt = prec == lbm.LBM_FP64 or base == lbm.LBM_BASE_LOCAL_REST
    for geom in (lbm.LBM_GEOM_CELL, lbm.LBM_GEOM_CELL_TABLE):
        g = lbm.Grid(case, precision=prec, offset_base=base, geometry=geom)
        assert g.info.table_kind == (2 if geom == lbm.LBM_GEOM_CELL and rebuilt else 1)
        g.init(u0)
        g.step(200)
        out.append((g.get_state()[0], g.moments()[2]))
        g.close()
    (Pa, Uta), (Pb, Utb) = out
    d_state = norm_rel(Pa, Pb)
    d_u = np.abs(Uta - Utb).max() / np.abs(Utb).max()
    say("prec", prec, "base", base, "rebuilt vs stored: state %.2e, Ut %.2e" % (d_state, d_u))
    # FP16 stores an 11-bit mantissa (unit roundoff 4.9e-4).  The two paths
    # form the same terms in different orders (FP64 differences of staged
    # tangents rounded once, against stored FP32 values), so their FP32
    # results differ by about one FP32 ulp per step; storing rounds such a
    # difference to a different FP16 value now and then, and each flip is a
    # full FP16 ulp of the offset.  Over 200 steps these flips add up to a few
    # 1e-3 of the peak velocity (4.8e-3 measured at the w rho0 base), the same
    # order as FP16's own error against the oracle (up to 2e-2 of the
    # characteristic speed in the parity tests); 1e-2 is twice the measured
    # figure and half that error bound.
    tol = {lbm.LBM_FP64: 1e-13, lbm.LBM_FP32: 2e-6, lbm.LBM_FP16: 1e-2}[prec]
    assert d_u <= tol
    if not rebuilt:
        assert np.array_equal(Pa, Pb)


def test_rebuilt_geometry_base_none_reads_stored_tables():
    """FP32 populations stored with no offset base (the particle numbers
    themselves) take the stored per-cell table whichever per-cell mode is
    asked for: the pulled sources move from a zero storage base to the cell's
    compute base by the table's FP64-rounded differences."""
    case = G.periodic_box(21, 40, 300, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    u0 = initial_velocity(case)
    out = []
    for geom in (lbm.LBM_GEOM_CELL, lbm.LBM_GEOM_CELL_TABLE):
        g = lbm.Grid(case, precision=lbm.LBM_FP32, offset_base=lbm.LBM_BASE_NONE, geometry=geom)
        assert g.info.table_kind == 1
        g.init(u0)
        g.step(200)
        out.append(g.get_state()[0])
        g.close()
    assert np.array_equal(out[0], out[1])


BASE_NONE_CASES = [c for c in CASES if c[0] in ("box_wobble_q21_wide", "eccentric_q21", "annulus_q21_moving",
                                                  "couette_q9")]


@pytest.mark.parametrize("name,case", BASE_NONE_CASES, ids=[c[0] for c in BASE_NONE_CASES])
def test_rebuilt_geometry_fp32_base_none_matches_oracle(name, case):
    """FP32 storage with no offset base on a per-cell path (the stored
    table): the state stays within the FP32 gate of the FP64 oracle (velocity
    within 1e-5 of the characteristic speed, particle number within 1e-6)."""
    g, o = pair(case, precision=lbm.LBM_FP32, geometry=lbm.LBM_GEOM_CELL, offset_base=lbm.LBM_BASE_NONE)
    assert g.info.table_kind == 1
    g.step(300)
    o.step(300)
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    geo = o.geometry()
    u = Ut[:, :1] * geo["g1"] + Ut[:, 1:] * geo["g2"]
    uo = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    err = np.abs(u - uo).max() / characteristic_speed(case, uo)
    say(name, "fp32 base none, rebuilt geometry: velocity err / U %.2e, m %.2e" % (err, norm_rel(m, mo)))
    assert err <= 1e-5
    assert norm_rel(m, mo) <= 1e-6
    # the state as stored and read back carries the mass the moments pass
    # sees (streaming permutes populations, so the totals agree)
    P, _ = g.get_state()
    assert abs(P.sum() - m.sum()) <= 1e-6 * m.sum()


def test_table_kind_selection():
    wob = G.periodic_box(21, 9, 11, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    ann = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8)
    assert lbm.Grid(wob).info.table_kind == 2
    assert lbm.Grid(ann).info.table_kind == 0
    assert lbm.Grid(ann, geometry=lbm.LBM_GEOM_CELL).info.table_kind == 2
    assert lbm.Grid(ann, geometry=lbm.LBM_GEOM_CELL_TABLE).info.table_kind == 1
    assert lbm.Grid(wob, geometry=lbm.LBM_GEOM_CELL_TABLE).info.table_kind == 1


@pytest.mark.parametrize("fuse", [0, lbm.LBM_BATCH_FUSE_LATTICES], ids=["groups", "fused"])
def test_rebuilt_geometry_in_batches(fuse):
    """Grids with rebuilt per-cell terms form their own launch group (or share
    the fused launch) and end exactly as they do alone."""
    cases = [G.periodic_box(21, 10, 150, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9),
             G.periodic_box(9, 12, 140, dx=1.0, dy=1.2, wobble=0.2, tau=0.8),
             G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8)]
    for prec in (lbm.LBM_FP64, lbm.LBM_FP32):
        alone = [lbm.Grid(c, precision=prec) for c in cases]
        batched = [lbm.Grid(c, precision=prec) for c in cases]
        for g, c in zip(alone + batched, cases + cases):
            g.init(initial_velocity(c))
        for g in alone:
            g.step(45)
        b = lbm.lbm_batch_create_ex([g.h for g in batched], fuse)
        groups = lbm.lbm_batch_groups(b)
        say("groups", groups)
        lbm.lbm_batch_step(b, 45)
        lbm.lbm_batch_destroy(b)
        for ga, gb in zip(alone, batched):
            assert np.array_equal(ga.get_state()[0], gb.get_state()[0])


def test_rebuilt_geometry_iterated_force():
    """Fixed-point passes of the force relation (iterations > 0) read the
    rebuilt Christoffel sums in every pass."""
    case = G.periodic_box(21, 10, 150, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    g, o = pair(case, iterations=2, geometry=lbm.LBM_GEOM_CELL)
    g.step(100)
    o.step(100)
    P, _ = g.get_state()
    err = norm_rel(to_oracle_state(P), o.get_state())
    say("iterated force, rebuilt geometry: state rel err %.2e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("prec,steps,tolu,tol1", [(lbm.LBM_FP64, 600, 1e-11, 1e-13), (lbm.LBM_FP32, 2000, 1e-5, 3e-6)],
                         ids=["fp64", "fp32"])
def test_rebuilt_geometry_full_size_annulus(prec, steps, tolu, tol1):
    """A 128 x 1024 annulus (R2 = 2 R1, cells of aspect 0.79 to 1.57) forced
    onto the per-cell path: every column is rebuilt from its own staged
    geometry (rotated copies of the same row, equal only to rounding), and the
    state still follows the oracle's exact theta-reduction.  In FP64 the
    columns' Christoffel sums, differences of neighbouring tangents, differ
    from the reduction's single column by rounding amplified by the 1/(r dtheta)
    of a difference (~1e-13 relative), hence 1e-11 of U against the reduction;
    the step's own arithmetic is then checked cell by cell against the
    oracle's step of the same state on the full grid.  (The 256 x 1024
    annulus, whose outer cells reach aspect 3.1, is unstable to the
    non-axisymmetric perturbations such rounding seeds, on the oracle as on
    the GPU; only its exactly theta-invariant form is stable.)"""
    case = G.circular_couette(21, 128, 1024, 128.0, u_inner=0.05, tau=0.8)
    g = lbm.Grid(case, precision=prec, geometry=lbm.LBM_GEOM_CELL)
    assert g.info.table_kind == 2
    g.init()
    g.step(steps)
    red = oracle.OracleGrid(G.circular_couette(21, 128, 1024, 128.0, u_inner=0.05, tau=0.8, n2=1))
    red.init(1.0)
    red.step(steps)
    m, U, Ut = g.moments()
    mo, Uo, Uto = red.moments()
    sdt = np.sin(case.meta["dtheta"])
    r_c = case.meta["centres"]
    uth = Ut.reshape(128, 1024, 2)[:, :, 1] * r_c[:, None] * sdt
    uth_o = Uto[:, 1] * r_c * sdt
    err = np.abs(uth - uth_o[:, None]).max()
    say("annulus 128x1024 rebuilt geometry prec", prec, "u_theta err / U %.2e" % (err / 0.05))
    assert err <= tolu * 0.05
    # the per-cell arithmetic itself, on the full grid's own geometry
    e1 = one_step_sampled(g, case)
    say("one-step sampled rel err %.2e" % e1)
    assert e1 <= tol1


def test_rebuilt_geometry_noflow_volume():
    """The "no flow" adjustment on the per-cell path gives the per-row path's
    volume J' (Sec. 3.1)."""
    case = G.circular_couette(21, 10, 80, 10.0, u_inner=0.05, tau=1.0)
    vols = []
    for geom in (lbm.LBM_GEOM_AUTO, lbm.LBM_GEOM_CELL):
        g = lbm.Grid(case, geometry=geom)
        steps = g.noflow_adjust(tol=1e-12, check_every=500)
        vols.append((steps, g.get_volume()))
    assert vols[0][0] == vols[1][0]
    assert norm_rel(vols[1][1], vols[0][1]) <= 1e-12


@pytest.mark.parametrize("prec", [lbm.LBM_FP64, lbm.LBM_FP32], ids=["fp64", "fp32"])
def test_rebuilt_geometry_checkpoint_resume(prec):
    """lbm_save / lbm_load on a grid with rebuilt per-cell terms: the restored
    grid continues as the original.  Loading re-forms the lagged force sums
    with the Christoffel sums of the stored per-cell table, equal to the
    rebuilt ones to rounding, so the two runs agree to rounding rather than
    bitwise."""
    case = G.eccentric_annulus(21, 16, 150, 16.0, 1.0, tau=1.0)
    a = lbm.Grid(case, precision=prec)
    assert a.info.table_kind == 2
    a.init()
    a.step(33)
    blob = a.save()
    b = lbm.Grid(case, precision=prec)
    b.load(blob)
    a.step(40)
    b.step(40)
    tol = 1e-13 if prec == lbm.LBM_FP64 else 1e-6
    d = norm_rel(b.get_state()[0], a.get_state()[0])
    say("checkpoint resume, rebuilt geometry, prec", prec, "state rel diff %.2e" % d)
    assert d <= tol
    assert b.info.step == a.info.step
