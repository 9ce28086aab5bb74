"""The paper's exact solutions (Sec. 3) and the oracle's convergence to them
under refinement (CPU only).  Flows are invariant along q2, so each run keeps
one periodic column continued with the true q2 step (exact for such states)."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact as ex
from paper_2301_01868_amd import grids as G
from steady import run_to_steady


def _d(f, r, h=1e-4):
    return (f(r + h) - f(r - h)) / (2 * h)


def _d2(f, r, h=1e-4):
    return (f(r + h) - 2 * f(r) + f(r - h)) / h ** 2


def test_exact_solutions_solve_their_equations():
    R1, R2, nu, T0 = 2.0, 5.0, 0.2, 2.0 / 3.0
    r = np.linspace(R1 + 0.1, R2 - 0.1, 7)
    # circular Couette: -u/r^2 + (1/r) d/dr (r du/dr) = 0, u(R_k) = Omega_k R_k
    Om1, Om2 = 0.03, -0.01
    u = lambda x: ex.circular_couette(x, R1, R2, Om1, Om2)
    assert np.allclose(-u(r) / r ** 2 + _d(u, r) / r + _d2(u, r), 0, atol=1e-6)
    assert abs(u(R1) - Om1 * R1) < 1e-14 and abs(u(R2) - Om2 * R2) < 1e-14
    # circular Poiseuille with acceleration K r: nu (...) + K r = 0, no slip
    K = 1e-3
    up = lambda x: ex.circular_poiseuille(x, R1, R2, K, nu)
    assert np.allclose(nu * (-up(r) / r ** 2 + _d(up, r) / r + _d2(up, r)) + K * r, 0, atol=1e-7)
    assert abs(up(R1)) < 1e-14 and abs(up(R2)) < 1e-13
    closed = K * (r ** 2 - R1 ** 2) * (R2 ** 2 - r ** 2) / (8 * nu * r)
    assert np.allclose(up(r), closed, rtol=1e-12)
    rr = np.linspace(R1, R2, 200001)
    assert abs(np.trapezoid(up(rr), rr) / (R2 - R1) - ex.circular_poiseuille_mean(R1, R2, K, nu)) < 1e-10
    # densities: d rho/dr = rho0 u^2 / (r T0) and the mass integral of Sec. 3.3
    for dens, vel in ((lambda x: ex.circular_couette_density(x, R1, R2, Om1, Om2, T0), u),
                      (lambda x: ex.circular_poiseuille_density(x, R1, R2, K, nu, T0), up)):
        assert np.allclose(_d(dens, r), vel(r) ** 2 / (r * T0), rtol=1e-6, atol=1e-12)
        assert abs(np.trapezoid(rr * dens(rr), rr) - (R2 ** 2 - R1 ** 2) / 2) < 1e-9
    # planar: linear Couette and parabolic Poiseuille
    X = np.linspace(0, 8, 9)
    assert np.allclose(ex.planar_couette(X, 8.0, -0.1, 0.0), 0.1 * (X / 8 - 1))   # U0 (x/l - 1), U0 = 0.1
    g = 1e-5
    pp = ex.planar_poiseuille(X, 8.0, g, nu)
    assert abs(pp[0]) < 1e-15 and abs(pp[-1]) < 1e-15
    assert np.allclose(nu * np.gradient(np.gradient(pp, X), X)[2:-2] + g, 0, atol=1e-12)
    assert abs(ex.planar_poiseuille_g(0.05, 8, nu) * 64 / (12 * nu) - 0.05) < 1e-15


def _table_rows():
    import os
    rows = []
    for ln in open(os.path.join(os.path.dirname(__file__), "golden", "parameter_tables.txt")):
        if ln.strip() and not ln.startswith("#"):
            rows.append(ln.split())
    return rows


def test_parameter_tables_regenerate():
    """nu = T0 (tau - 1/2), Ma = U / sqrt(T0), Re = U N / nu, planar Poiseuille
    g = 12 nu U / N^2, Fr = U / sqrt(g N), circular Couette Omega1 = U / M with
    M = N_r / 10 (NCR = 11), N_theta = N_r 2 pi R1 / (R2 - R1)."""
    for r in _table_rows():
        tab = r[0]
        q = 9 if tab.endswith("9") else 21
        T0 = 1 / 3 if q == 9 else 2 / 3
        tau = float(r[1])
        nu = ex.nu_lat(T0, tau)
        if tab.startswith("CC"):
            Nr, Nt, Om, nu_p, U, Ma, Re = int(r[2]), int(r[3]), *map(float, r[4:])
            assert abs(nu - nu_p) < 6e-4
            M = Nr / 10
            U_exact = Re * nu / Nr
            assert abs(Om - U_exact / M) / Om < 6e-3
            assert abs(ex.mach(U, T0) - Ma) < 2e-3
            assert abs(Nr * 2 * math.pi * M / Nr - Nt) / Nt < 0.01     # the tables round N_theta
            continue
        N = int(r[2])
        U, nu_p, Ma, Re = map(float, r[3:7])
        assert abs(nu - nu_p) < 6e-4
        U_exact = Re * nu / N          # the printed U is rounded; Re is exact
        assert abs(U_exact - U) / U < 0.02
        assert abs(ex.mach(U_exact, T0) - Ma) < 6e-4
        if tab.startswith("PP"):
            g, Fr = float(r[7]), float(r[8])
            gg = ex.planar_poiseuille_g(U_exact, N, nu)
            assert abs(gg - g) / g < 6e-3
            assert abs(U_exact / math.sqrt(gg * N) - Fr) < 0.051


def _planar_err(case, sol, iters=0, tol=1e-11):
    o = oracle.OracleGrid(case)
    o.init(1.0)
    o.set_iterations(iters)
    run_to_steady(o, tol=tol)
    m, U, Ut = o.moments()
    u = o.physical_velocity(Ut)[:, 1]
    return np.abs(u - sol).max()


def test_planar_couette_q9_uniform_is_exact():
    for N in (8, 16):
        c = G.planar_couette(9, G.faces_uniform(N), u_wall=0.05)
        err = _planar_err(c, ex.planar_couette(c.meta["centres"], N, 0.0, 0.05), tol=1e-14)
        assert err < 1e-13


def test_planar_poiseuille_q9_uniform_second_order():
    errs = []
    for N in (8, 16, 32):
        nu = G.viscosity(9, 1.0)
        g = 12 * nu * 0.05 / N ** 2
        c = G.planar_poiseuille(9, G.faces_uniform(N), g=g)
        sol = ex.planar_poiseuille(c.meta["centres"], N, g, nu)
        errs.append(_planar_err(c, sol) / sol.max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


@pytest.mark.parametrize("q,iters", [(21, 0), (9, 1)])
def test_planar_contracting_grid_converges(q, iters):
    """CR = 0.4 linear contraction (App. C): error against the exact profiles
    falls under refinement (D2Q9 with one fixed-point force pass)."""
    for prob in ("couette", "poiseuille"):
        errs = []
        for N in (8, 16, 32):
            f = G.faces_linear(N, 0.4)
            nu = G.viscosity(q, 1.0)
            if prob == "couette":
                c = G.planar_couette(q, f, u_wall=0.05)
                sol, scale = ex.planar_couette(c.meta["centres"], N, 0.0, 0.05), 0.05
            else:
                g = 12 * nu * 0.05 / N ** 2
                c = G.planar_poiseuille(q, f, g=g)
                sol = ex.planar_poiseuille(c.meta["centres"], N, g, nu)
                scale = sol.max()
            errs.append(_planar_err(c, sol, iters) / scale)
        assert errs[0] > errs[1] > errs[2], (prob, errs)
        assert errs[0] / errs[2] > 3.0 and errs[2] < 0.05, (prob, errs)


def _circ(q, Nr, prob, NCR=2.0, tau=1.0):
    M = Nr / (NCR - 1.0)
    nu = G.viscosity(q, tau)
    if prob == "couette":
        c = G.circular_couette(q, Nr, 4 * Nr, M, u_inner=0.05, tau=tau, n2=1)
        sol = lambda r: ex.circular_couette(r, M, M + Nr, 0.05 / M, 0.0)
    else:
        g2 = G.poiseuille_g2_for_peak(Nr, 4 * Nr, M, nu, 0.05)
        c = G.circular_poiseuille(q, Nr, 4 * Nr, M, g2=g2, tau=tau, n2=1)
        K = c.meta["K"]
        sol = lambda r: ex.circular_poiseuille(r, M, M + Nr, K, nu)
    return c, sol


@pytest.mark.parametrize("prob", ["couette", "poiseuille"])
def test_circular_q21_converges(prob):
    errs = []
    for Nr in (8, 16, 32):
        c, sol = _circ(21, Nr, prob)
        o = oracle.OracleGrid(c)
        o.init(1.0)
        run_to_steady(o, tol=1e-11)
        m, U, Ut = o.moments()
        r = c.meta["centres"]
        uth = Ut[:, 1] * r * math.sin(c.meta["dtheta"])     # App. D: u_theta = U^2 sin(dtheta) r
        errs.append(np.abs(uth - sol(r)).max() / 0.05)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.02


def test_q9_polar_period2_mode_grows():
    """D2Q9's neutral period-2 mode (eigenvalue -1 on a uniform grid) is pushed
    outside the unit circle by the lagged inertial force on polar grids.  On
    the theta-reduced circular Couette flow (NCR = 2, Nr = 8, tau = 1) the
    period-2 component of the state, N(t) - 2 N(t+1) + N(t+2), keeps growing
    where D2Q21 converges (test_circular_q21_converges), so the D2Q9 circular
    flows overflow instead of settling on a wrong profile."""
    c, _ = _circ(9, 8, "couette")
    o = oracle.OracleGrid(c)
    o.init(1.0)

    def period2():
        P0 = o.get_state().copy()
        o.step(1)
        P1 = o.get_state().copy()
        o.step(1)
        P2 = o.get_state().copy()
        return np.abs(P0 - 2 * P1 + P2).max()

    o.step(1000)
    a = period2()
    o.step(248)
    b = period2()
    assert np.isfinite(b) and b > 1.5 * a > 0, (a, b)
