"""Continuous-batching server (needs an MI355X): every solve converges to the
same result alone and inside a stream of other solves."""
import numpy as np
import pytest

from gpu_util import say
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm
from paper_2301_01868_amd import serve

pytestmark = pytest.mark.gpu


def test_alone_equals_mixed():
    """Requests admitted into batches that are already running (the budget
    holds about two and a half of the largest request, so most requests wait
    for earlier ones to retire) end bitwise as they do alone, after the same
    number of steps."""
    trace = serve.make_trace(seed=7, rate=400.0, duration=0.05, n_min=16, n_max=32, tol=1e-6)
    say("trace", len(trace), "requests")
    assert len(trace) >= 10
    one = max(serve.request_bytes(r.case, lbm.LBM_FP32) for r in trace)
    srv = serve.Server(hbm_budget=int(2.5 * one), check_every=100)
    info = srv.run(trace, realtime=False)
    s = serve.summarize(trace, info["makespan"])
    say("mixed", s, "admission rounds", [r.admit_round for r in trace])
    assert s["converged"] + s["unstable"] == len(trace)
    late = [r for r in trace if r.admit_round > 0]
    assert len(late) >= 5
    # the first requests (admitted at round 0) and every late-admitted one
    for r in trace[:3] + late:
        alone = serve.Request(rid=r.rid, arrival=0.0, case=r.case, tol=r.tol)
        serve.Server(hbm_budget=64 << 20, check_every=100).run([alone], realtime=False)
        assert alone.status == r.status and alone.steps == r.steps, r.rid
        if r.status == "converged":
            assert np.array_equal(alone.result["Ut"], r.result["Ut"]), r.rid


def test_admission_respects_budget():
    trace = serve.make_trace(seed=8, rate=400.0, duration=0.03, n_min=32, n_max=48, tol=1e-5)
    one = max(serve.request_bytes(r.case, lbm.LBM_FP32) for r in trace)
    srv = serve.Server(hbm_budget=2 * one, check_every=100)
    srv.run(trace, realtime=False)
    assert all(r.status in ("converged", "unstable") for r in trace)


def test_unstable_request_is_isolated():
    """A request whose state overflows (the 16 x 128 channel stretched by 1.02
    per cell, whose wall cells leave the lattice's stable band and overflow
    within about 200 steps) is retired as unstable; the requests running
    beside it in the same batches converge to exactly the results they get
    alone."""
    trace = serve.make_trace(seed=9, rate=400.0, duration=0.02, n_min=16, n_max=24, tol=1e-6)
    bad = serve.Request(rid=len(trace), arrival=0.0, case=G.workload_planar_poiseuille(128, 0.6), tol=1e-6)
    mixed = trace + [bad]
    serve.Server(hbm_budget=64 << 20, check_every=100).run(mixed, realtime=False)
    say("statuses", [r.status for r in mixed])
    assert bad.status == "unstable"
    for r in trace:
        alone = serve.Request(rid=r.rid, arrival=0.0, case=r.case, tol=r.tol)
        serve.Server(hbm_budget=64 << 20, check_every=100).run([alone], realtime=False)
        assert alone.status == r.status and alone.steps == r.steps
        if r.status == "converged":
            assert np.array_equal(alone.result["Ut"], r.result["Ut"])
