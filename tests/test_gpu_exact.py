"""The circular flows of Sec. 3.3-3.4 run to steady state on the GPU (needs an
MI355X): circular Couette against u_theta = A r + B / r and circular
Poiseuille against the paper's profile, on the exact theta-reduction of the
annulus (one periodic column continued with the true angular step), under
refinement, with and without the "no flow" volume adjustment.  The library's
steady states are also compared with the oracle's."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import say
from oracle import exact as ex
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm
from steady import run_to_steady

pytestmark = pytest.mark.gpu


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


def _gpu_steady(g, tol=1e-10, K=1000, max_steps=400000):
    g.residual()
    steps, R = 0, math.inf
    while steps < max_steps:
        g.step(K)
        steps += K
        R = g.residual().residual
        if R < tol:
            break
    return steps, R


def _u_theta(c, Ut):
    return Ut[:, 1] * c.meta["centres"] * math.sin(c.meta["dtheta"])   # App. D: u_theta = U^2 sin(dtheta) r


@pytest.mark.parametrize("prob", ["couette", "poiseuille"])
def test_circular_flows_converge_to_exact_profiles(prob):
    """Errors against the exact profile fall under refinement, and equal the
    FP64 oracle's at every resolution.  (The oracle gives Couette errors
    falling at about order 1.5, the moving wall's specular source with its
    correction being the lower-order boundary, and Poiseuille errors at about
    order 1.9.)"""
    errs, errs_o = [], []
    for Nr in (16, 32, 64):
        c, sol = _circ(21, Nr, prob)
        r = c.meta["centres"]
        g = lbm.Grid(c, precision=lbm.LBM_FP64)
        g.init()
        steps, R = _gpu_steady(g)
        assert R < 1e-10, (Nr, R)
        m, U, Ut = g.moments()
        errs.append(np.abs(_u_theta(c, Ut) - sol(r)).max() / 0.05)
        o = oracle.OracleGrid(c)
        o.init(1.0)
        run_to_steady(o, tol=1e-10, K=1000)
        mo, Uo, Uto = o.moments()
        errs_o.append(np.abs(_u_theta(c, Uto) - sol(r)).max() / 0.05)
        say(prob, "Nr", Nr, "steps", steps, "max |u - exact| / U %.4e (oracle %.4e)" % (errs[-1], errs_o[-1]))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[0] / errs[2] > 2.5 and errs[2] < 0.01, errs
    assert np.allclose(errs, errs_o, rtol=1e-6), (errs, errs_o)


def test_noflow_volume_leaves_the_steady_velocity_unchanged():
    """The "no flow" adjustment replaces J by J' = m_nf / rho0.  The step works
    in particle numbers, where J cancels, so the steady velocity is the same
    and only the reported density changes: rho0 everywhere in the no-flow
    state, against a non-uniform density with the geometric J."""
    c, sol = _circ(21, 16, "couette")
    a = lbm.Grid(c, precision=lbm.LBM_FP64)
    a.init()
    _gpu_steady(a)
    b = lbm.Grid(c, precision=lbm.LBM_FP64)
    b.noflow_adjust(tol=1e-12, check_every=1000)
    b.init()
    _gpu_steady(b)
    Ua = a.moments()[2]
    Ub = b.moments()[2]
    assert np.abs(Ua - Ub).max() <= 1e-9 * np.abs(Ua).max()
    nf = lbm.Grid(c.no_flow(), precision=lbm.LBM_FP64)
    nf.noflow_adjust(tol=1e-12, check_every=1000)
    nf.init()
    _gpu_steady(nf, tol=1e-12)
    m = nf.moments()[0]
    rho = m / nf.get_volume()
    geo = nf.geometry()[:, 0]
    say("no-flow density range with J' %.2e, with J %.2e" % (np.ptp(rho), np.ptp(m / geo)))
    assert np.abs(rho - c.rho0).max() < 1e-9
    assert np.ptp(m / geo) > 1e-4


@pytest.mark.parametrize("prob", ["couette", "poiseuille"])
def test_circular_steady_state_equals_oracle(prob):
    c, sol = _circ(21, 16, prob)
    g = lbm.Grid(c, precision=lbm.LBM_FP64)
    g.init()
    steps, R = _gpu_steady(g, K=500)
    o = oracle.OracleGrid(c)
    o.init(1.0)
    n_o, R_o = run_to_steady(o, tol=1e-10, K=500)
    assert steps == n_o
    m, U, Ut = g.moments()
    mo, Uo, Uto = o.moments()
    assert np.abs(Ut - Uto).max() <= 1e-11 * np.abs(Uto).max()
