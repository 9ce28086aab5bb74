"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X)."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import characteristic_speed, norm_rel, pair, say, side_to_oracle, to_oracle_state
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu


def _cases():
    yield "couette_q9_nonequilateral", G.workload_planar_couette_q9()
    yield "annulus_q21_moving", G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    yield "channel_cr_q21_ragged", G.planar_couette(21, G.faces_linear(14, 0.35), n2=70, u_wall=0.04, moving="lo",
                                                     tau=0.7).replace(accel=(0.0, 2e-6))
    yield "box_wobble_q21_cells", G.periodic_box(21, 9, 11, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9)
    yield "box_q9", G.periodic_box(9, 7, 66, dx=1.0, dy=1.4, tau=0.6)
    yield "annulus_poiseuille_q9", G.circular_poiseuille(9, 6, 80, 10.0, g2=1e-4, tau=0.7)
    yield "narrow_q21", G.planar_couette(21, G.faces_uniform(3), n2=5, u_wall=0.03, tau=1.0)
    yield "eccentric_q21_nonorthogonal", G.eccentric_annulus(21, 10, 90, 12.0, 1.0, tau=1.0)


CASES = list(_cases())


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_stream_map_bitexact(name, case):
    g = lbm.Grid(case)
    o = oracle.OracleGrid(case)
    sc, sd, wl = g.stream_map()
    osc, osd, owl = o.stream_map()
    assert (sc == osc).all() and (sd == osd).all() and (wl == owl).all()


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_geometry_precompute(name, case):
    g = lbm.Grid(case)
    o = oracle.OracleGrid(case)
    geo = g.geometry()
    ref = o.geometry()
    q = case.q
    assert np.allclose(geo[:, 0], ref["J"], rtol=1e-13, atol=0)
    assert np.abs(geo[:, 1:4] - ref["G"]).max() <= 1e-12 * np.abs(ref["G"]).max()
    Ap = geo[:, 4:].reshape(-1, q, 2)
    assert np.abs(Ap - ref["Aplus"]).max() <= 1e-12 * max(1.0, np.abs(ref["Aplus"]).max())
    info = g.info
    expect_rows = case.meta.get("family") in ("planar", "polar") or case.meta.get("wobble", 1) == 0
    assert bool(info.row_tables) == bool(expect_rows)


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_fp64_trajectory(name, case):
    """FP64 GPU step vs the oracle from the same initial state, many steps.

    The first step's lagged force reads N'(q, -1) = the initial state (a
    reading: the paper gives no value before the first step).  Both sides
    implement that reading; no value the paper prints fixes it, so this part
    of the trajectory is "parity unpinned" beyond the oracle's rest-state pin
    on uniform metrics."""
    steps = 5000 if name.startswith("couette_q9") else 300
    g, o = pair(case)
    g.step(steps)
    o.step(steps)
    P, side = g.get_state()
    Po = o.get_state()
    err = norm_rel(to_oracle_state(P), Po)
    say(name, "state rel err", err)
    assert err <= 1e-12
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    assert norm_rel(m, mo) <= 1e-12
    assert np.abs(Ut - Uto).max() <= 1e-12 * max(np.abs(Uto).max(), 1e-3)
    assert np.abs(U - Uo).max() <= 1e-12 * max(np.abs(Uo).max(), 1e-3)


def test_fp64_iterated_force():
    case = G.planar_couette(9, G.faces_linear(12, 0.4), n2=3, u_wall=0.05, tau=0.8)
    g, o = pair(case, iterations=2)
    g.step(500)
    o.step(500)
    P, _ = g.get_state()
    assert norm_rel(to_oracle_state(P), o.get_state()) <= 1e-12


def _iter_cases():
    # D2Q21 per-row tables with moving walls on both sides; n2 = 100 takes only
    # the general pull path, n2 = 200 also the unwrapped fast path (n2 >= 131).
    # The wider annulus has R1 = 30 (cells of aspect 0.94 to 1.32, inside the
    # lattice's stable band): with R1 = 20 (aspect 0.63 at the inner wall) the
    # oracle and the GPU part exponentially from the inner wall, with or
    # without fixed-point passes (4e-8 after 300 steps), and with R1 = 10 the
    # state overflows within 10 steps on both.
    yield "annulus_q21_moving_12x100", G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    yield "annulus_q21_moving_12x200", G.circular_couette(21, 12, 200, 30.0, u_inner=0.05, u_outer=-0.02, tau=0.8)


ITER_CASES = list(_iter_cases())


@pytest.mark.parametrize("iters", [1, 2])
@pytest.mark.parametrize("name,case", ITER_CASES, ids=[c[0] for c in ITER_CASES])
def test_iterated_force_q21_rows(name, case, iters):
    """Fixed-point passes of the implicit force relation (Sec. 2, the
    iterative alternative to the one-step lag under Eq. compo-constr) on the
    D2Q21 per-row kernels: FP64 state within 1e-12 of the oracle's iterated
    step after 300 steps; FP32 physical velocity within 1e-5 of the
    characteristic speed."""
    g, o = pair(case, iterations=iters)
    assert g.info.row_tables == 1
    g.step(300)
    o.step(300)
    P, _ = g.get_state()
    err = norm_rel(to_oracle_state(P), o.get_state())
    say(name, "iterations", iters, "fp64 state rel err %.2e" % err)
    assert err <= 1e-12
    g32 = lbm.Grid(case, precision=lbm.LBM_FP32, iterations=iters)
    g32.init()
    g32.step(300)
    m, U, Ut = g32.moments()
    mo, Uo, Uto = o.moments()
    geo = o.geometry()
    u = Ut[:, :1] * geo["g1"] + Ut[:, 1:] * geo["g2"]
    uo = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    Uc = characteristic_speed(case, uo)
    e32 = np.abs(u - uo).max() / Uc
    say(name, "iterations", iters, "fp32 velocity err / U %.2e" % e32)
    assert e32 <= 1e-5
    assert norm_rel(m, mo) <= 1e-6


def test_residual_value_matches_its_definition():
    """lbm_residual's R against the same definition formed from the oracle's
    moments, |m Ut(t) - m Ut(t - K)|_2 / (K |m Ut(t)|_2) over interior cells.
    The definition is this library's reading (the paper judges steady state by
    energy and angular momentum and defines no residual), so the value is
    "parity unpinned": both sides implement the reading, nothing in the paper
    fixes it."""
    from steady import residual as ref_residual
    case = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    g, o = pair(case)
    g.residual(check=False)
    K = 50
    rs = []
    prev = None
    for _ in range(3):
        g.step(K)
        o.step(K)
        R = g.residual(check=False).residual
        mo, Uo, Uto = o.moments()
        cur = mo[:, None] * Uto
        if prev is not None:
            rs.append((R, ref_residual(prev, cur, K)))
        prev = cur
    for R, Ro in rs:
        say("residual gpu %.6e oracle-formed %.6e" % (R, Ro))
        assert abs(R - Ro) <= 1e-10 * Ro


@pytest.mark.parametrize("name,case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_one_step_from_gpu_state(name, case):
    """The oracle's single step from the GPU's state (populations and wall
    side state) reproduces the GPU's next state."""
    g, o = pair(case)
    g.step(37)
    P0, side0 = g.get_state()
    o.set_state(to_oracle_state(P0))
    m_s, u_s = side_to_oracle(side0, case.n1, case.n2)
    o.set_side(np.nan_to_num(m_s), np.nan_to_num(u_s))
    g.step(1)
    P1, _ = g.get_state()
    o.step(1)
    assert norm_rel(to_oracle_state(P1), o.get_state()) <= 1e-13


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_fp32_velocity_within_tolerance(name, case):
    """FP32 offset storage + FP32 arithmetic: velocity within 1e-5 of the
    characteristic speed of the FP64 oracle after the same number of steps."""
    steps = 2000 if name.startswith("couette_q9") else 300
    g, o = pair(case, precision=lbm.LBM_FP32)
    g.step(steps)
    o.step(steps)
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    geo = o.geometry()
    u = Ut[:, :1] * geo["g1"] + Ut[:, 1:] * geo["g2"]
    uo = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    Uc = characteristic_speed(case, uo)
    err = np.abs(u - uo).max()
    say(name, "fp32 velocity err / U", err / Uc)
    assert err <= 1e-5 * Uc
    assert norm_rel(m, mo) <= 1e-6


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_fp16_velocity_error_stated(name, case):
    """FP16 storage (per-direction scaled offsets, FP32 arithmetic): the error
    against the FP64 oracle is measured and reported (an 11-bit mantissa on
    the stored offsets); it must stay within 2e-2 of the characteristic speed."""
    steps = 2000 if name.startswith("couette_q9") else 300
    g, o = pair(case, precision=lbm.LBM_FP16)
    g.step(steps)
    o.step(steps)
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    geo = o.geometry()
    u = Ut[:, :1] * geo["g1"] + Ut[:, 1:] * geo["g2"]
    uo = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    Uc = characteristic_speed(case, uo)
    err = np.abs(u - uo).max() / Uc
    say(name, "fp16 velocity err / U", err)
    assert err <= 2e-2


def test_moments_residual_and_mass():
    case = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8)
    g, o = pair(case)
    r0 = g.residual()
    g.step(200)
    o.step(200)
    r = g.residual()
    mo, Uo, Uto = o.moments()
    assert abs(r.mass - mo.sum()) <= 1e-12 * mo.sum()
    assert abs(r.mass_rel_drift) < 1e-13
    geo = o.geometry()
    u = Uto[:, :1] * geo["g1"] + Uto[:, 1:] * geo["g2"]
    ke = 0.5 * (mo * (u ** 2).sum(1)).sum()
    xc = case.X[case.halo:-case.halo, case.halo:-case.halo].ravel()
    yc = case.Y[case.halo:-case.halo, case.halo:-case.halo].ravel()
    am = (mo * (xc * u[:, 1] - yc * u[:, 0])).sum()
    assert abs(r.kinetic_energy - ke) <= 1e-11 * ke
    assert abs(r.angular_momentum - am) <= 1e-11 * abs(am)
    assert r.bad_cells == 0 and math.isfinite(r.residual) and r.residual > 0
    assert not math.isfinite(r0.residual) or r0.residual >= 0


def test_noflow_adjust_matches_oracle_procedure():
    case = G.circular_couette(21, 10, 80, 10.0, u_inner=0.05, tau=1.0)
    g = lbm.Grid(case)
    steps = g.noflow_adjust(tol=1e-12, check_every=500)
    say("no-flow steps", steps)
    o = oracle.OracleGrid(case.no_flow())
    o.init(1.0)
    o.step(steps)
    mo, _, _ = o.moments()
    # J' = m_nf / rho0 from the same number of no-flow steps
    assert norm_rel(g.get_volume(), mo / case.rho0) <= 1e-11


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_physical_velocity_matches_oracle(name, case):
    """Ut^i g_i per cell (the velocity the paper's profiles show)."""
    g, o = pair(case)
    g.step(40)
    o.step(40)
    u = g.physical_velocity()
    mo, Uo, Uto = o.moments()
    uo = o.physical_velocity(Uto)
    assert np.abs(u - uo).max() <= 1e-12 * max(np.abs(uo).max(), 1e-3)
