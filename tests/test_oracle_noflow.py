"""The "no flow" volume adjustment of Sec. 3.1 applied with the oracle (CPU only)."""
import numpy as np

import oracle
from paper_2301_01868_amd import grids as G
from steady import run_to_steady


def test_no_flow_adjustment_gives_uniform_density():
    """J' = J rho_nf / rho0 = m_nf / rho0 from the no-flow steady state; a
    no-flow run initialised with J' then reports rho = rho0 everywhere, and the
    total volume (hence the total mass) is unchanged."""
    case = G.circular_couette(21, 16, 64, 16.0, u_inner=0.05, tau=1.0, n2=1)
    nf = oracle.OracleGrid(case.no_flow())
    nf.init(1.0)
    run_to_steady(nf, tol=1e-13)
    m_nf, _, _ = nf.moments()
    J = nf.geometry()["J"]
    rho_nf = m_nf / J
    assert np.abs(rho_nf - 1).max() > 1e-4         # curvilinear grids: not uniform before
    Jp = m_nf / 1.0
    assert abs(Jp.sum() - J.sum()) / J.sum() < 1e-13
    again = oracle.OracleGrid(case.no_flow())
    again.set_volume(Jp)
    again.init(1.0)
    run_to_steady(again, tol=1e-13)
    m2, _, _ = again.moments()
    assert np.abs(m2 / Jp - 1.0).max() < 1e-9
