"""The 64-annulus ensemble at full size, batched in FP32, against the exact
theta-reduction of each instance on the oracle (needs an MI355X).

Some instances of the ensemble are linearly unstable for the method itself:
the FP64 oracle amplifies a 1e-9 relative perturbation of the start state
instead of damping it (D2Q21 on cells far from equilateral, or close to
tau = 1/2).  On those, any two computations that round differently part
exponentially, so an FP32-vs-FP64 bound at a fixed step count says nothing
about the kernel; parity is asserted on the instances the oracle shows to be
stable, and for the others the test checks that the GPU and the oracle agree
on a blow-up where the oracle has one within the horizon."""
import numpy as np
import pytest

import oracle
from gpu_util import say
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu

STEPS = 100


def _reduced(c):
    M, Nr, Nt = c.meta["M"], c.meta["Nr"], c.meta["Ntheta"]
    if c.meta["problem"] == "circular_couette":
        return G.circular_couette(c.q, Nr, Nt, M, u_inner=0.05, tau=c.tau, n2=1)
    return G.circular_poiseuille(c.q, Nr, Nt, M, g2=c.meta["g2"], tau=c.tau, n2=1)


def _oracle_stable(rc, seed, horizon=400, rel=1e-9):
    """Perturbation test on the oracle: run the start state and a copy
    perturbed by `rel` (relative, seeded) side by side; the instance counts as
    stable when the difference stays finite and does not grow by more than 10x
    from STEPS to `horizon` steps (damped instances oscillate within about 2x
    while decaying; a growing mode amplifies it by orders of magnitude)."""
    a = oracle.OracleGrid(rc)
    a.init(1.0)
    b = oracle.OracleGrid(rc)
    b.init(1.0)
    s = b.get_state()
    s = s * (1.0 + rel * np.random.default_rng(seed).standard_normal(s.shape))
    b.set_state(s)
    a.step(STEPS)
    b.step(STEPS)
    d0 = np.abs(a.get_state() - b.get_state()).max()
    a.step(horizon - STEPS)
    b.step(horizon - STEPS)
    d1 = np.abs(a.get_state() - b.get_state()).max()
    return bool(np.isfinite(d0) and np.isfinite(d1) and d1 <= 10.0 * d0), d0, d1


_ORACLE = {}

# instances the oracle's perturbation test finds linearly unstable (all D2Q21:
# four with cells of aspect 0.54-0.60 at the inner wall that overflow within
# 100 steps, and instance 17 at tau 0.562 with aspect 2.5, which grows about
# 20x per 100 steps)
UNSTABLE = [17, 26, 28, 47, 62]


def _oracle_state(k, c):
    """Oracle moments (m, U, Ut) of instance k after STEPS steps on its exact
    theta-reduction, and its stability class (cached: the tests share them)."""
    if k not in _ORACLE:
        rc = _reduced(c)
        o = oracle.OracleGrid(rc)
        o.init(1.0)
        o.step(STEPS)
        _ORACLE[k] = (o.moments(), o.get_state(), _oracle_stable(rc, seed=k))
    return _ORACLE[k]


def _run_batched(cases, prec):
    grids = [lbm.Grid(c, precision=prec) for c in cases]
    for g in grids:
        g.init()
    b = lbm.lbm_batch_create([g.h for g in grids])
    lbm.lbm_batch_step(b, STEPS)
    recs = lbm.lbm_batch_residuals(b, len(grids))
    lbm.lbm_batch_destroy(b)
    return grids, recs


def _column(g, c):
    """Moments of column 0 (every column is equal: asserted by the callers)."""
    m, U, Ut = g.moments()
    return m.reshape(c.n1, c.n2), U.reshape(c.n1, c.n2, 2), Ut.reshape(c.n1, c.n2, 2)


def test_ensemble_batched_fp16_error_stated():
    """FP16 storage (offsets scaled by 1/w per direction plane) on the whole
    ensemble: the error against the oracle is printed per instance and
    bounded loosely; FP16 rounding (about 5e-4 relative) sets it."""
    cases = G.workload_ensemble()
    grids, recs = _run_batched(cases, lbm.LBM_FP16)
    errs = []
    for k, (c, g, r) in enumerate(zip(cases, grids, recs)):
        (mo, Uo, Uto), _, (stable, d0, d1) = _oracle_state(k, c)
        if not stable:
            continue
        assert r.bad_cells == 0, k
        m, U, Ut = _column(g, c)
        errs.append(np.abs((Ut[:, 0, 1] - Uto[:, 1]) * c.meta["centres"] * np.sin(c.meta["dtheta"])).max() / 0.05)
    errs = np.array(errs)
    say("ensemble FP16: %d stable instances, u_theta err / U median %.2e, max %.2e" % (len(errs), np.median(errs), errs.max()))
    assert errs.max() <= 5e-3


def test_ensemble_batched_fp32_vs_reduced_oracle():
    """FP32 populations, batched, 100 steps: on every stable instance the
    physical velocity (radial Ut^1 |g_1| with |g_1| = 1 on these uniform
    radial grids, and azimuthal Ut^2 r sin(dtheta)) within 1e-5 of the wall
    speed, and the particle number m within 1e-6 relative, of the oracle's
    exact theta-reduction; the unstable set is exactly the oracle's."""
    cases = G.workload_ensemble()
    grids, recs = _run_batched(cases, lbm.LBM_FP32)
    worst = {"u_theta": 0.0, "u_r": 0.0, "m": 0.0}
    checked, unstable = 0, []
    for k, (c, g, r) in enumerate(zip(cases, grids, recs)):
        (mo, Uo, Uto), _, (stable, d0, d1) = _oracle_state(k, c)
        ok_o = np.isfinite(Uto).all()
        assert ok_o == (r.bad_cells == 0), k
        if not stable:
            unstable.append(k)
            say("instance %d unstable in the oracle (Q%d, %dx%d, tau %.3f): perturbation %.1e -> %.1e"
                % (k, c.q, c.n1, c.n2, c.tau, d0, d1))
            continue
        m, U, Ut = _column(g, c)
        # theta-invariance is exact on the GPU (row tables)
        assert (Ut == Ut[:, :1, :]).all() and (m == m[:, :1]).all()
        r_c = c.meta["centres"]
        sdt = np.sin(c.meta["dtheta"])
        e_th = np.abs((Ut[:, 0, 1] - Uto[:, 1]) * r_c * sdt).max() / 0.05
        e_r = np.abs(Ut[:, 0, 0] - Uto[:, 0]).max() / 0.05
        e_m = np.abs(m[:, 0] - mo).max() / np.abs(mo).max()
        for key, e in (("u_theta", e_th), ("u_r", e_r), ("m", e_m)):
            worst[key] = max(worst[key], e)
        checked += 1
        assert e_th <= 1e-5 and e_r <= 1e-5, (k, e_th, e_r)
        assert e_m <= 1e-6, (k, e_m)
    say("ensemble FP32: %d stable instances, worst u_theta / U %.2e, u_r / U %.2e, m %.2e; oracle-unstable %s"
        % (checked, worst["u_theta"], worst["u_r"], worst["m"], unstable))
    assert unstable == UNSTABLE
    assert checked == len(cases) - len(UNSTABLE) == 59


def test_ensemble_batched_fp64_vs_reduced_oracle():
    """FP64 populations, batched, 100 steps: on every stable instance the
    state (all Q directions of column 0) within 1e-12 norm-relative of the
    oracle's exact theta-reduction, and the physical velocity within 1e-12 of
    the larger of the wall speed and the oracle's largest speed (the FP64
    trajectory reading: a per-step rounding difference set by the
    populations, not by the current speed)."""
    cases = G.workload_ensemble()
    grids, recs = _run_batched(cases, lbm.LBM_FP64)
    worst_s, worst_u, checked = 0.0, 0.0, 0
    for k, (c, g, r) in enumerate(zip(cases, grids, recs)):
        (mo, Uo, Uto), Po, (stable, d0, d1) = _oracle_state(k, c)
        assert np.isfinite(Uto).all() == (r.bad_cells == 0), k
        if not stable:
            continue
        P, _ = g.get_state()
        assert (P == P[:, :, :1]).all()
        col = np.ascontiguousarray(P[:, :, 0].T)      # [row][Q], the reduction's layout
        e_s = np.abs(col - Po).max() / np.abs(Po).max()
        m, U, Ut = _column(g, c)
        uth = Ut[:, 0, 1] * c.meta["centres"] * np.sin(c.meta["dtheta"])
        uth_o = Uto[:, 1] * c.meta["centres"] * np.sin(c.meta["dtheta"])
        e_u = np.abs(uth - uth_o).max() / max(np.abs(uth_o).max(), 0.05)
        worst_s, worst_u = max(worst_s, e_s), max(worst_u, e_u)
        checked += 1
        assert e_s <= 1e-12 and e_u <= 1e-12, (k, e_s, e_u)
    say("ensemble FP64: %d stable instances, worst state rel %.2e, u_theta %.2e" % (checked, worst_s, worst_u))
    assert checked == 59
