"""Continuous-batching server (needs an MI355X): every solve converges to the
same result alone and inside a stream of other solves."""
import numpy as np
import pytest

from gpu_util import say
from paper_2301_01868_amd import lbm
from paper_2301_01868_amd import serve

pytestmark = pytest.mark.gpu


def test_alone_equals_mixed():
    trace = serve.make_trace(seed=7, rate=400.0, duration=0.05, n_min=16, n_max=32, tol=1e-6)
    say("trace", len(trace), "requests")
    assert len(trace) >= 10
    srv = serve.Server(hbm_budget=64 << 20, check_every=100)
    info = srv.run(trace, realtime=False)
    s = serve.summarize(trace, info["makespan"])
    say("mixed", s)
    assert s["converged"] + s["unstable"] == len(trace)
    for r in trace[:5]:
        alone = serve.Request(rid=r.rid, arrival=0.0, case=r.case, tol=r.tol)
        serve.Server(hbm_budget=64 << 20, check_every=100).run([alone], realtime=False)
        assert alone.status == r.status and alone.steps == r.steps
        if r.status == "converged":
            Ua, Um = alone.result["Ut"], r.result["Ut"]
            U = max(np.abs(Um).max(), 1e-3)
            assert np.abs(Ua - Um).max() <= 1e-5 * U
            assert np.array_equal(Ua, Um)


def test_admission_respects_budget():
    trace = serve.make_trace(seed=8, rate=400.0, duration=0.03, n_min=32, n_max=48, tol=1e-5)
    one = max(serve.request_bytes(r.case, lbm.LBM_FP32) for r in trace)
    srv = serve.Server(hbm_budget=2 * one, check_every=100)
    srv.run(trace, realtime=False)
    assert all(r.status in ("converged", "unstable") for r in trace)
