"""Serving: a continuous-batching request loop over the C ABI.

Requests are steady-state solves: a grid, a lattice, a relaxation time and a
residual tolerance.  They arrive over time; the server keeps every admitted
solve's populations resident in HBM, admits new solves between rounds as
device memory frees up (an HBM budget), advances all resident solves together
with one fused batched launch per step (HIP-graph captured), checks
each solve's residual every round, and retires solves that converged, turned
unstable, stalled (residual no longer falling) or reached the step limit.
The sequential baseline replays the same trace one solve at a time, first come
first served, in FP64.

Latency of a request = completion time - arrival time (queueing included).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import grids as G
from . import lbm


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    case: G.Case
    tol: float = 1e-8
    # filled by a run
    start: float = math.nan
    finish: float = math.nan
    steps: int = 0
    residual: float = math.nan
    status: str = "pending"
    result: dict = field(default_factory=dict)
    best: float = math.inf        # lowest residual that halved the previous best
    best_step: int = 0            # step count at which `best` was reached
    admit_round: int = -1         # server round before which the request was admitted


def check_progress(r, res, max_steps, stall_steps):
    """Record a residual check of request `r` after its steps were counted;
    return its final status, or None while it keeps running.  A solve whose
    residual has not halved within `stall_steps` steps is stalled: a
    converging solve halves it every ln 2 times its slowest decay time, while
    a solve caught in a saturated unsteady state (an instability of the
    scheme that does not overflow) keeps it level."""
    r.residual = res.residual
    if res.bad_cells > 0:
        return "unstable"
    if res.residual < r.tol:
        return "converged"
    if res.residual < 0.5 * r.best:
        r.best, r.best_step = res.residual, r.steps
    if r.steps - r.best_step >= stall_steps:
        return "stalled"
    if r.steps >= max_steps:
        return "max_steps"
    return None


def request_bytes(case, precision):
    """Device bytes a solve holds: two population buffers plus the FP64
    per-cell arrays and tables (an upper estimate used for admission)."""
    s = 4 if precision == lbm.LBM_FP32 else 8
    pitch = case.n2 if case.n2 < 64 else (case.n2 + 63) // 64 * 64
    pops = 2 * case.q * case.n1 * pitch * s
    per_cell = 8 * (11 + 5 + 2) + 8 * case.q
    halo = 16 * (case.n1 + 2 * case.halo) * (case.n2 + 2 * case.halo)
    return pops + per_cell * case.ncell + halo + (1 << 20)


def make_trace(seed=2301_01869, rate=50.0, duration=60.0, n_min=16, n_max=128, tol=1e-8):
    """Poisson arrivals; each request is a steady-state solve drawn from the
    paper's problem families: planar Couette or Poiseuille on a uniform
    channel (D2Q9 or D2Q21), or circular Couette on an annulus (D2Q21) with
    R2/R1 in [1.5, 3]; wall-normal resolution log-uniform in [n_min, n_max];
    tau in [0.55, 1]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        N = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) / 2)) * 2
        tau = float(rng.uniform(0.55, 1.0))
        fam = int(rng.integers(3))
        q = 21 if (fam == 2 or rng.random() < 0.5) else 9
        if fam == 0:
            case = G.planar_couette(q, G.faces_uniform(N), n2=N, u_wall=0.05, tau=tau)
        elif fam == 1:
            nu = G.viscosity(q, tau)
            case = G.planar_poiseuille(q, G.faces_uniform(N), n2=N, g=8 * nu * 0.05 / N ** 2, tau=tau)
        else:
            ratio = float(rng.uniform(1.5, 3.0))
            case = G.circular_couette(21, N, 4 * N, N / (ratio - 1.0), u_inner=0.05, tau=tau)
        reqs.append(Request(rid=len(reqs), arrival=t, case=case, tol=tol))
    return reqs


class Server:
    def __init__(self, hbm_budget=8 << 30, check_every=200, precision=lbm.LBM_FP32, max_steps=2_000_000,
                 stream=None, stall_steps=200_000):
        self.budget = hbm_budget
        self.K = check_every
        self.precision = precision
        self.max_steps = max_steps
        self.stall_steps = stall_steps
        self.stream = stream

    def run(self, requests, realtime=True):
        """Serve the trace.  With realtime=True arrivals are honoured against the
        wall clock; otherwise every request is available at time 0."""
        pending = sorted(requests, key=lambda r: r.arrival)
        active = {}          # rid -> (request, Grid)
        used = 0
        batch = None
        dirty = True
        t0 = time.perf_counter()
        k = 0
        rounds = 0
        while k < len(pending) or active:
            now = time.perf_counter() - t0
            # admit every arrived request that fits the budget (first come first served)
            while k < len(pending) and (not realtime or pending[k].arrival <= now):
                r = pending[k]
                need = request_bytes(r.case, self.precision)
                if used + need > self.budget and active:
                    break
                g = lbm.Grid(r.case, precision=self.precision, stream=self.stream)
                g.init()
                r.start = time.perf_counter() - t0
                r.status = "running"
                r.admit_round = rounds
                active[r.rid] = (r, g, need)
                used += need
                k += 1
                dirty = True
            if not active:
                if k < len(pending):
                    time.sleep(max(0.0, pending[k].arrival - (time.perf_counter() - t0)))
                continue
            if dirty:
                if batch is not None:
                    lbm.lbm_batch_destroy(batch)
                # one fused launch per step for both lattices: the resident solves
                # are small and their steps launch-bound
                batch = lbm.lbm_batch_create_ex([g.h for (_, g, _) in active.values()], lbm.LBM_BATCH_FUSE_LATTICES)
                dirty = False
            lbm.lbm_batch_step(batch, self.K)
            rounds += 1
            done = []
            items = list(active.items())
            recs = lbm.lbm_batch_residuals(batch, len(items))
            for (rid, (r, g, need)), res in zip(items, recs):
                r.steps += self.K
                st = check_progress(r, res, self.max_steps, self.stall_steps)
                if st is not None:
                    r.status = st
                    done.append(rid)
            if done:
                now = time.perf_counter() - t0
                # the batch goes before the grids it holds (a grid may own its stream)
                lbm.lbm_batch_destroy(batch)
                batch = None
                for rid in done:
                    r, g, need = active.pop(rid)
                    r.finish = now
                    m, U, Ut = g.moments()
                    r.result = {"Ut": Ut}
                    g.close()
                    used -= need
                dirty = True
        if batch is not None:
            lbm.lbm_batch_destroy(batch)
        return {"makespan": time.perf_counter() - t0, "rounds": rounds}


def run_sequential(requests, precision=lbm.LBM_FP64, check_every=200, max_steps=2_000_000, stream=None,
                   realtime=True, stall_steps=200_000):
    """Plain one-solve-at-a-time stepping, first come first served."""
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        g = lbm.Grid(r.case, precision=precision, stream=stream)
        g.init()
        r.start = time.perf_counter() - t0
        while True:
            g.step(check_every)
            r.steps += check_every
            st = check_progress(r, g.residual(check=False), max_steps, stall_steps)
            if st is not None:
                r.status = st
                break
        m, U, Ut = g.moments()
        r.result = {"Ut": Ut}
        r.finish = time.perf_counter() - t0
        g.close()
    return {"makespan": time.perf_counter() - t0}


def summarize(requests, makespan):
    lat = np.array([r.finish - r.arrival for r in requests if math.isfinite(r.finish)])
    ok = [r for r in requests if r.status == "converged"]
    lups = sum(r.steps * r.case.ncell for r in requests)
    return {"requests": len(requests), "converged": len(ok),
            "unstable": sum(r.status == "unstable" for r in requests),
            "stalled": sum(r.status == "stalled" for r in requests),
            "max_steps": sum(r.status == "max_steps" for r in requests),
            "solves_per_s": len(ok) / makespan if makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "makespan_s": makespan, "glups": lups / makespan / 1e9 if makespan > 0 else 0.0}
