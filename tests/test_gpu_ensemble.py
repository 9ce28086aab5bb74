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


def _oracle_state(k, c):
    """Oracle u^theta-related moments of instance k after STEPS steps, and its
    stability class (cached: the FP32 and FP16 tests share them)."""
    if k not in _ORACLE:
        rc = _reduced(c)
        o = oracle.OracleGrid(rc)
        o.init(1.0)
        o.step(STEPS)
        mo, Uo, Uto = o.moments()
        _ORACLE[k] = (Uto, _oracle_stable(rc, seed=k))
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


def test_ensemble_batched_fp16_error_stated():
    """FP16 storage (offsets scaled by 1/w per direction plane) on the whole
    ensemble: the error against the oracle is printed per instance and
    bounded loosely; FP16 rounding (about 5e-4 relative) sets it."""
    cases = G.workload_ensemble()
    grids, recs = _run_batched(cases, lbm.LBM_FP16)
    errs = []
    for k, (c, g, r) in enumerate(zip(cases, grids, recs)):
        Uto, (stable, d0, d1) = _oracle_state(k, c)
        if not stable:
            continue
        assert r.bad_cells == 0, k
        m, U, Ut = g.moments()
        col = Ut.reshape(c.n1, c.n2, 2)[:, 0]
        errs.append(np.abs((col[:, 1] - Uto[:, 1]) * c.meta["centres"] * np.sin(c.meta["dtheta"])).max() / 0.05)
    errs = np.array(errs)
    say("ensemble FP16: %d stable instances, u_theta err / U median %.2e, max %.2e" % (len(errs), np.median(errs), errs.max()))
    assert errs.max() <= 5e-3


def test_ensemble_batched_fp32_vs_reduced_oracle():
    cases = G.workload_ensemble()
    grids, recs = _run_batched(cases, lbm.LBM_FP32)
    worst, checked, unstable = 0.0, 0, []
    for k, (c, g, r) in enumerate(zip(cases, grids, recs)):
        Uto, (stable, d0, d1) = _oracle_state(k, c)
        ok_o = np.isfinite(Uto).all()
        assert ok_o == (r.bad_cells == 0), k
        if not stable:
            unstable.append(k)
            say("instance %d unstable in the oracle (Q%d, %dx%d, tau %.3f): perturbation %.1e -> %.1e"
                % (k, c.q, c.n1, c.n2, c.tau, d0, d1))
            continue
        m, U, Ut = g.moments()
        col = Ut.reshape(c.n1, c.n2, 2)[:, 0]
        # theta-invariance is exact on the GPU (row tables)
        assert (Ut.reshape(c.n1, c.n2, 2) == col[:, None, :]).all()
        r_c = c.meta["centres"]
        sdt = np.sin(c.meta["dtheta"])
        err = np.abs((col[:, 1] - Uto[:, 1]) * r_c * sdt).max() / 0.05
        worst = max(worst, err)
        checked += 1
        assert err <= 1e-5, (k, err)
    say("ensemble: %d stable instances, worst u_theta err / U %.2e; oracle-unstable %s" % (checked, worst, unstable))
    assert checked >= 48
