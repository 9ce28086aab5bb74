"""The serving loop's retirement rule (host logic, CPU only)."""
import math
from types import SimpleNamespace

from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import serve


def _req():
    return serve.Request(rid=0, arrival=0.0, case=G.planar_couette(9, G.faces_uniform(8)), tol=1e-8)


def _run(residuals, K=200, max_steps=10**9, stall=2000):
    r = _req()
    for R in residuals:
        r.steps += K
        st = serve.check_progress(r, SimpleNamespace(residual=R, bad_cells=0), max_steps, stall)
        if st is not None:
            return st, r.steps
    return None, r.steps


def test_converging_solve_is_never_stalled():
    # halves every 1000 steps (5 checks), slower than it could and still fine
    res = [1e-3 * 0.5 ** (k / 5.0) for k in range(200)]
    st, steps = _run(res)
    assert st == "converged"
    assert res[steps // 200 - 1] < 1e-8


def test_saturated_solve_is_stalled():
    res = [3e-5 * (1.0 + 0.3 * math.sin(k)) for k in range(1000)]
    st, steps = _run(res)
    assert st == "stalled"
    assert steps <= 2000 + 2 * 200


def test_unstable_and_step_limit():
    r = _req()
    r.steps = 200
    assert serve.check_progress(r, SimpleNamespace(residual=1e-3, bad_cells=5), 10**9, 10**6) == "unstable"
    st, steps = _run([1e-3 * 0.5 ** (k / 5.0) for k in range(200)], max_steps=1000)
    assert (st, steps) == ("max_steps", 1000)


def test_slow_solves_get_fp64_storage():
    from paper_2301_01868_amd import lbm
    srv = object.__new__(serve.Server)          # the policy alone: no streams or pool needed
    srv.precision, srv.fp64_above = lbm.LBM_FP32, 10_000.0
    fast = serve.Request(rid=0, arrival=0.0, case=G.planar_couette(9, G.faces_uniform(8), n2=4), tol=1e-8)
    slow = serve.Request(rid=1, arrival=0.0, case=G.planar_couette(9, G.faces_uniform(256), n2=4), tol=1e-8)
    assert serve.slow_decay_steps(fast.case) < 10_000 < serve.slow_decay_steps(slow.case)
    assert srv.precision_of(fast) == lbm.LBM_FP32 and srv.precision_of(slow) == lbm.LBM_FP64
    # admission charges the larger population buffers
    assert serve.request_bytes(slow.case, lbm.LBM_FP64) > serve.request_bytes(slow.case, lbm.LBM_FP32)
    srv.fp64_above = None
    assert srv.precision_of(slow) == lbm.LBM_FP32
