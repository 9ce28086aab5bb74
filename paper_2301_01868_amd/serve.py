"""Serving: a continuous-batching request loop over the C ABI.

Requests are steady-state solves: a grid, a lattice, a relaxation time and a
residual tolerance.  They arrive over time.  The server keeps every admitted
solve's populations resident in HBM and advances all of them together: one
fused launch per step over a flattened tile table, replayed from an
instantiated HIP graph.  Each round it

1. launches the next ``check_every`` steps of the batch (asynchronously),
2. while those run, creates and initialises the requests that have arrived and
   fit the HBM budget, on a setup stream (their set-up overlaps the steps),
3. reads every member's residual (the one synchronisation of the round),
4. retires solves that converged, turned unstable, stalled (residual no longer
   falling) or reached their step limit, and
5. updates the batch's membership in place (the library rewrites the tile and
   instance tables and the graph's kernel nodes; nothing is rebuilt).

Device memory of the grids comes from PyTorch's caching allocator through the
library's allocator hooks, so admitting and retiring solves allocates and
frees nothing on the device once the pool is warm.

The sequential baseline replays requests one solve at a time, first come
first served, in FP64.  Latency of a request = completion time - arrival time
(queueing + service).
"""
from __future__ import annotations

import ctypes as ct
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
    pred_steps: int = 0     # predicted steps to the tolerance (see predict_steps)
    # filled by a run
    start: float = math.nan       # admission time (set-up done, joins the next round)
    finish: float = math.nan
    steps: int = 0
    residual: float = math.nan
    status: str = "pending"
    result: dict = field(default_factory=dict)
    best: float = math.inf        # lowest residual that halved the previous best
    best_step: int = 0            # step count at which `best` was reached
    admit_round: int = -1         # server round before which the request was admitted
    precision: int = -1           # population storage the server chose


def slow_decay_steps(case):
    """Decay time, in steps, of the slowest viscous mode across the channel or
    gap: L^2 / (pi^2 nu) with L the wall-normal extent in lattice units."""
    L = float(case.meta.get("l", case.n1))
    return L * L / (math.pi ** 2 * G.viscosity(case.q, case.tau))


def predict_steps(case, tol):
    """Steps until the residual (the per-step relative change of the velocity)
    falls below tol, for a start from rest: the slowest mode's amplitude
    exp(-t / T) changes by exp(-t / T) / T per step, so t = T ln(1 / (T tol))."""
    T = slow_decay_steps(case)
    return int(max(1000.0, T * max(1.0, math.log(1.0 / (T * tol)))))


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


def limits(r, max_steps, stall_steps):
    """Step limit and stall window of a request: at least the server's, and
    scaled with the request's own slowest decay time (a solve of 512 cells
    across at tau 0.55 needs millions of steps and halves its residual only
    every 0.7 million)."""
    T = slow_decay_steps(r.case)
    return max(max_steps, 4 * r.pred_steps), max(stall_steps, int(4.0 * T))


def request_bytes(case, precision):
    """Device bytes a solve holds: two population buffers plus the FP64
    per-cell arrays and tables (an upper estimate used for admission)."""
    s = {lbm.LBM_FP16: 2, lbm.LBM_FP32: 4}.get(precision, 8)
    pitch = case.n2 if case.n2 < 64 else (case.n2 + 63) // 64 * 64
    pops = 2 * case.q * case.n1 * pitch * s
    per_cell = 8 * (11 + 5 + 2) + 8 * case.q
    halo = 16 * (case.n1 + 2 * case.halo) * (case.n2 + 2 * case.halo)
    return pops + per_cell * case.ncell + halo + (1 << 20)


# ---------------------------------------------------------------------------
# request traces
# ---------------------------------------------------------------------------
FAMILIES = ("planar_couette", "planar_poiseuille", "circular_couette", "circular_poiseuille")


def _stretch_ratio(N, ratio=1.02, min_wall=0.75):
    """Geometric stretching from both walls at `ratio`, reduced (bisection) so
    that the wall cell stays at least min_wall of the mean step: finer wall
    cells leave the lattice's stable range and overflow."""
    def wall(rho):
        K = N // 2
        return 1.0 if rho == 1.0 else K * (rho - 1.0) / (rho ** K - 1.0)
    if wall(ratio) >= min_wall:
        return ratio
    lo, hi = 1.0, ratio
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if wall(mid) >= min_wall else (lo, mid)
    return lo


def draw_params(rng, n_min=16, n_max=512):
    """One request's parameters: family, wall-normal resolution N
    (log-uniform over [n_min, n_max], even), N x 4N cells, tau ~ U(0.55, 1),
    lattice (D2Q9 or D2Q21 with equal odds on the planar families; D2Q21 on
    the annuli, where D2Q9 carries a growing period-2 mode), and for the
    annuli R2/R1 ~ U(1.5, 4)."""
    N = max(4, int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max))) / 2)) * 2)
    tau = float(rng.uniform(0.55, 1.0))
    fam = FAMILIES[int(rng.integers(len(FAMILIES)))]
    q = 21 if (fam.startswith("circular") or rng.random() < 0.5) else 9
    ratio = float(rng.uniform(1.5, 4.0))
    return dict(family=fam, N=N, n2=4 * N, tau=tau, q=q, ratio=ratio)


def build_case(p):
    """The Case of a parameter draw: planar Couette on a uniform channel with
    cells twice as long as wide (dx = 2 dy, the D2Q9 Couette workload's
    cells); planar Poiseuille on a channel stretched from both walls
    (ratio 1.02, reduced where the wall cell would fall below 0.75) with the
    force set for a peak speed of 0.05; circular Couette (inner wall at 0.05)
    and circular Poiseuille (peak 0.05) on uniform polar grids."""
    N, n2, q, tau = p["N"], p["n2"], p["q"], p["tau"]
    nu = G.viscosity(q, tau)
    if p["family"] == "planar_couette":
        c = G.planar_couette(q, G.faces_uniform(N), n2=n2, d_per=2.0, u_wall=0.05, tau=tau)
    elif p["family"] == "planar_poiseuille":
        rho = 1.0 if q == 9 else _stretch_ratio(N)
        c = G.planar_poiseuille(q, G.faces_geometric(N, rho), n2=n2, g=8.0 * nu * 0.05 / N ** 2, tau=tau)
        c.meta.update(ratio=rho)
    else:
        M = N / (p["ratio"] - 1.0)
        if p["family"] == "circular_couette":
            c = G.circular_couette(q, N, n2, M, u_inner=0.05, tau=tau)
        else:
            c = G.circular_poiseuille(q, N, n2, M, g2=G.poiseuille_g2_for_peak(N, n2, M, nu, 0.05), tau=tau)
        c.meta.update(ratio=p["ratio"])
    c.meta.update(l=float(N))
    return c


def make_trace(seed=2301_01869, rate=50.0, duration=60.0, n_min=16, n_max=512, tol=1e-8, n_requests=None):
    """Poisson arrivals at `rate` per second for `duration` seconds (or the
    first n_requests arrivals), each request drawn by draw_params."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if n_requests is None and t > duration:
            break
        p = draw_params(rng, n_min, n_max)
        case = build_case(p)
        case.meta.update(draw=p)
        reqs.append(Request(rid=len(reqs), arrival=t, case=case, tol=tol, pred_steps=predict_steps(case, tol)))
        if n_requests is not None and len(reqs) >= n_requests:
            break
    return reqs


def mean_predicted_lu(seed=1, n_min=16, n_max=512, tol=1e-8, samples=20000):
    """Mean predicted lattice updates per request of the trace distribution
    (Monte Carlo over draw_params; no grids are built)."""
    rng = np.random.default_rng(seed)
    tot = 0.0
    for _ in range(samples):
        p = draw_params(rng, n_min, n_max)
        T = p["N"] ** 2 / (math.pi ** 2 * G.viscosity(p["q"], p["tau"]))
        steps = max(1000.0, T * max(1.0, math.log(1.0 / (T * tol))))
        tot += steps * p["N"] * p["n2"]
    return tot / samples


# ---------------------------------------------------------------------------
# device memory from PyTorch's caching allocator
# ---------------------------------------------------------------------------
class TorchPool:
    """lbm_allocator backed by torch.cuda's caching allocator on `stream`
    (a torch.cuda.Stream): blocks freed by a retired grid are reused by the
    next admitted one without a hipFree (which would synchronise the device).
    Blocks are tied to the stream they were allocated on; the server frees a
    grid only after every use of it, on any stream, has completed."""

    _ALLOC = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
    _FREE = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)

    def __init__(self, stream, device=0):
        import torch

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            except Exception:        # out of memory: the library reports LBM_ENOMEM
                return None

        def _free(ptr, ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)

        self._cbs = (self._ALLOC(_alloc), self._FREE(_free))
        self.desc = lbm.lbm_allocator(ct.cast(self._cbs[0], ct.c_void_p), ct.cast(self._cbs[1], ct.c_void_p), None)


def _raw(stream):
    return None if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)


# ---------------------------------------------------------------------------
# the server
# ---------------------------------------------------------------------------
class Server:
    """Continuous batching of steady-state solves.  `stream` is the stream
    the batch runs on and `setup_stream` the one new grids are created on
    (torch.cuda.Stream objects; both made here when None).  `pool`: use the
    torch caching allocator for grid memory.  `fp64_above`: a slowest decay
    time (steps) above which a request runs with FP64 populations instead of
    `precision`: FP32 storage rounds the state every step, and for the
    slowest mode that rounding adds up over its decay time, so slowly
    converging solves need FP64 to keep their steady velocity within 1e-5 of
    the speed scale (None: every request in `precision`)."""

    def __init__(self, hbm_budget=8 << 30, check_every=256, precision=lbm.LBM_FP32, max_steps=2_000_000,
                 stream=None, stall_steps=200_000, setup_stream=None, pool=True, fp64_above=None):
        import torch
        self.budget = hbm_budget
        self.K = check_every
        self.precision = precision
        self.max_steps = max_steps
        self.stall_steps = stall_steps
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.setup_stream = setup_stream if setup_stream is not None else torch.cuda.Stream()
        self.pool = TorchPool(self.setup_stream) if pool else None
        self.fp64_above = fp64_above
        self.stats = {}

    def precision_of(self, r):
        if self.fp64_above is not None and slow_decay_steps(r.case) > self.fp64_above:
            return lbm.LBM_FP64
        return self.precision

    def _admit(self, r, rounds, t0):
        r.precision = self.precision_of(r)
        g = lbm.Grid(r.case, precision=r.precision, stream=_raw(self.setup_stream),
                     alloc=None if self.pool is None else self.pool.desc)
        g.init()
        # queued set-up work stays ordered before the grid's first step
        g.set_stream(_raw(self.stream))
        r.start = time.perf_counter() - t0
        r.status = "running"
        r.admit_round = rounds
        return g

    def run(self, requests, realtime=True, stop_after=None, progress=None):
        """Serve the trace.  With realtime=True arrivals are honoured against the
        wall clock; otherwise every request is available at time 0.
        stop_after (seconds) ends the run early, leaving unfinished requests
        as they are (capacity measurements).  progress(text) is called about
        every 20 s with the run's state."""
        pending = sorted(requests, key=lambda r: r.arrival)
        active = []          # [(request, Grid, bytes, max_steps, stall_steps)]
        used = 0
        batch = None
        t0 = time.perf_counter()
        k = 0
        rounds = 0
        lu = 0
        t_setup = t_check = t_retire = 0.0
        peak = 0
        finished = 0
        t_note = t0
        try:
            while k < len(pending) or active:
                if progress is not None and time.perf_counter() - t_note > 20.0:
                    t_note = time.perf_counter()
                    progress("t %.0f s: %d admitted, %d resident, %d finished, %.3g lattice updates"
                             % (t_note - t0, k, len(active), finished, lu))
                if stop_after is not None and time.perf_counter() - t0 > stop_after:
                    break
                # 1. the round's steps run while the host admits
                if active:
                    lbm.lbm_batch_step(batch, self.K)
                    lu += self.K * sum(r.case.ncell for (r, *_rest) in active)
                # 2. admissions (first come first served, within the budget)
                ts = time.perf_counter()
                joined = []
                now = ts - t0
                while k < len(pending) and (not realtime or pending[k].arrival <= now):
                    r = pending[k]
                    need = request_bytes(r.case, self.precision_of(r))
                    if used + need > self.budget and (active or joined):
                        break
                    g = self._admit(r, rounds, t0)
                    ms, st = limits(r, self.max_steps, self.stall_steps)
                    joined.append((r, g, need, ms, st))
                    used += need
                    k += 1
                t_setup += time.perf_counter() - ts
                # 3. residuals of the members that stepped this round
                done = []
                if active:
                    tc = time.perf_counter()
                    recs = lbm.lbm_batch_residuals(batch, len(active))
                    t_check += time.perf_counter() - tc
                    for item, res in zip(active, recs):
                        r = item[0]
                        r.steps += self.K
                        stt = check_progress(r, res, item[3], item[4])
                        if stt is not None:
                            r.status = stt
                            done.append(item)
                    rounds += 1
                # 5. membership for the next round, updated in place
                if done or joined:
                    active = [a for a in active if not any(a is d for d in done)] + joined
                    handles = [a[1].h for a in active]
                    if batch is None:
                        if handles:
                            batch = lbm.lbm_batch_create_ex(handles, lbm.LBM_BATCH_FUSE_LATTICES)
                    else:
                        lbm.lbm_batch_update(batch, handles)
                    peak = max(peak, len(active))
                # 4. the retired grids have left the batch: read them out and release them
                if done:
                    tr = time.perf_counter()
                    now = tr - t0
                    for (r, g, need, _, _) in done:
                        finished += 1
                        r.finish = now
                        m, U, Ut = g.moments()
                        r.result = {"Ut": Ut, "u": g.physical_velocity()}
                        g.close()
                        used -= need
                    t_retire += time.perf_counter() - tr
                if not active and k < len(pending) and realtime:
                    time.sleep(max(0.0, pending[k].arrival - (time.perf_counter() - t0)))
        finally:
            if batch is not None:
                lbm.lbm_batch_destroy(batch)
            for (r, g, *_rest) in active:
                g.close()
        elapsed = time.perf_counter() - t0
        self.stats = {"makespan": elapsed, "rounds": rounds, "lattice_updates": lu,
                      "glups": lu / elapsed / 1e9 if elapsed > 0 else 0.0, "setup_s": t_setup, "check_s": t_check,
                      "retire_s": t_retire, "peak_resident": peak}
        return self.stats


def run_sequential(requests, precision=lbm.LBM_FP64, check_every=256, max_steps=2_000_000, stream=None,
                   realtime=True, stall_steps=200_000, progress=None):
    """Plain one-solve-at-a-time stepping, first come first served: one grid,
    check_every steps (graph launches), one residual check, repeat.
    progress(text) is called after each request."""
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        g = lbm.Grid(r.case, precision=precision, stream=_raw(stream))
        g.init()
        r.start = time.perf_counter() - t0
        ms, st = limits(r, max_steps, stall_steps)
        while True:
            g.step(check_every)
            r.steps += check_every
            stt = check_progress(r, g.residual(check=False), ms, st)
            if stt is not None:
                r.status = stt
                break
        m, U, Ut = g.moments()
        r.result = {"Ut": Ut, "u": g.physical_velocity()}
        r.finish = time.perf_counter() - t0
        g.close()
        if progress is not None:
            progress("sequential: request %d (%s, N %d) %s after %d steps, %.1f s"
                     % (r.rid, r.case.meta.get("problem"), r.case.n1, r.status, r.steps, r.finish - r.start))
    return {"makespan": time.perf_counter() - t0}


def _pct(a, p):
    return float(np.percentile(a, p)) if len(a) else None


def summarize(requests, makespan):
    fin = [r for r in requests if math.isfinite(r.finish)]
    lat = np.array([r.finish - r.arrival for r in fin])
    queue = np.array([r.start - r.arrival for r in fin])
    serv = np.array([r.finish - r.start for r in fin])
    ok = [r for r in requests if r.status == "converged"]
    lups = sum(r.steps * r.case.ncell for r in requests)
    return {"requests": len(requests), "converged": len(ok),
            "unstable": sum(r.status == "unstable" for r in requests),
            "stalled": sum(r.status == "stalled" for r in requests),
            "max_steps": sum(r.status == "max_steps" for r in requests),
            "unfinished": len(requests) - len(fin),
            "solves_per_s": len(ok) / makespan if makespan > 0 else 0.0,
            "p50_latency_s": _pct(lat, 50), "p99_latency_s": _pct(lat, 99),
            "p50_queue_s": _pct(queue, 50), "p99_queue_s": _pct(queue, 99),
            "p50_service_s": _pct(serv, 50), "p99_service_s": _pct(serv, 99),
            "makespan_s": makespan, "lattice_updates": lups,
            "glups": lups / makespan / 1e9 if makespan > 0 else 0.0}
