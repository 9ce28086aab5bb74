"""Helpers shared by the GPU parity tests (test infrastructure)."""
import sys

import numpy as np

import oracle
from paper_2301_01868_amd import lbm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_oracle_state(P):
    """[Q][n1][n2] -> [cell][Q]"""
    q = P.shape[0]
    return np.ascontiguousarray(P.reshape(q, -1).T)


def side_to_oracle(side, n1, n2):
    """[2 walls][2 fields][hw][n2] -> full per-cell (m, Ut^2) arrays (wall rows filled)."""
    hw = side.shape[2]
    m = np.full((n1, n2), np.nan)
    u = np.full((n1, n2), np.nan)
    for k in range(hw):
        if k < n1:
            m[k], u[k] = side[0, 0, k], side[0, 1, k]
    for k in range(hw):
        i = n1 - 1 - k
        if i >= 0 and np.isfinite(side[1, 0, k]).all() and (side[1, 0, k] != 0).any():
            m[i], u[i] = side[1, 0, k], side[1, 1, k]
    return m.ravel(), u.ravel()


def norm_rel(a, b):
    d = np.abs(a - b).max()
    s = np.abs(b).max()
    return d / s if s > 0 else d


def initial_velocity(case):
    """Smooth contravariant start field for doubly periodic boxes (a shear
    wave along q2 varying along q1 plus a weaker transverse wave); None
    (rest) for wall-bounded cases."""
    if not case.periodic1:
        return None
    i = np.arange(case.n1)[:, None] + 0.5
    j = np.arange(case.n2)[None, :] + 0.5
    u = np.zeros((case.n1, case.n2, 2))
    u[..., 1] = 0.03 * np.sin(2 * np.pi * i / case.n1) + 0 * j
    u[..., 0] = 0.01 * np.cos(2 * np.pi * j / case.n2) + 0 * i
    return u.reshape(-1, 2)


def characteristic_speed(case, u_now):
    """Velocity scale of a case: its physical wall speeds, the amplitude of the
    start field, or the current maximum, whichever is largest."""
    cand = [np.abs(u_now).max(), 1e-3]
    for k in ("u_wall", "u_inner", "u_outer"):
        if k in case.meta:
            cand.append(abs(case.meta[k]))
    if case.periodic1:
        cand.append(0.03)          # amplitude of initial_velocity()
    return max(cand)


def pair(case, precision=lbm.LBM_FP64, iterations=0, **kw):
    """GPU grid and oracle grid of the same case, both initialised alike
    (rest, or a smooth wave on doubly periodic boxes)."""
    say("case", case.meta.get("problem", case.meta.get("family")), "q", case.q, "n1", case.n1, "n2", case.n2,
        "prec", precision, "iters", iterations)
    g = lbm.Grid(case, precision=precision, iterations=iterations, **kw)
    o = oracle.OracleGrid(case)
    o.set_iterations(iterations)
    u0 = initial_velocity(case)
    g.init(u0)
    o.init(case.rho0, u0)
    return g, o


def one_step_sampled(g, case, nsample=1500, seed=0, iterations=0):
    """One GPU step from the grid's current state against the oracle's step of
    the same state on sampled cells (every wall-adjacent row plus random
    interior cells); max relative difference.  `iterations` must be the
    grid's fixed-point force passes."""
    P0, side0 = g.get_state()
    o = oracle.OracleGrid(case)
    o.set_iterations(iterations)
    o.set_state(to_oracle_state(P0))
    del P0
    m_s, u_s = side_to_oracle(side0, case.n1, case.n2)
    o.set_side(np.nan_to_num(m_s), np.nan_to_num(u_s))
    del m_s, u_s
    rng = np.random.default_rng(seed)
    # every wall-adjacent row plus random interior cells
    rows = list(range(min(4, case.n1))) + list(range(max(0, case.n1 - 4), case.n1))
    cells = [r * case.n2 + int(rng.integers(case.n2)) for r in rows]
    cells += list(rng.choice(case.ncell, nsample, replace=False))
    cells = np.array(sorted(set(cells)), dtype=np.int32)
    ref = o.step_cells(cells)
    del o
    g.step(1)
    P1, _ = g.get_state()
    got = P1.reshape(P1.shape[0], -1)[:, cells].T
    return np.abs(got - ref).max() / np.abs(ref).max()
