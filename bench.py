"""Throughput benchmark of the curvilinear lattice Boltzmann step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                [--geometry auto|cell|cell_table] [--iterations K] [--no-fp64] [--no-fp16] [--no-3d]
                [--no-large] [--no-cpu]
python bench.py --serve [--load F | --rate R] [--requests N] [--seq-sample K] [--no-sequential]

FP32 populations give the headline figure; the same workload is then timed
with FP64 and FP16 populations (reported under "fp64" and "fp16"), one
single 4096 x 16384 annulus with FP32 populations (a 5.6 GB buffer, under
"single_grid_fp32") and the 3D step (under "d3q39_fp64").

A step is one application of the whole fused update (pull streaming with the
wall sources, moments, lagged inertial force, equilibrium, momentum-flux and
curvilinear corrections, BGK, store) to every cell of the workload.  Inputs
(the grid geometry and the populations) are resident in HBM before the timed
region; only HIP graph launches of the step kernel run inside it.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published

# sources that define the step kernel and its launch; a recorded traffic figure
# is used only while their hash matches the one it was measured with
STEP_SOURCES = ["paper_2301_01868_amd/csrc/lbm_kernels.hpp", "paper_2301_01868_amd/csrc/lbm_lattice.hpp",
                "paper_2301_01868_amd/csrc/lbm_lib.hip", "paper_2301_01868_amd/build.py"]


def step_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for f in sources or STEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


STEP3_SOURCES = ["paper_2301_01868_amd/csrc/lbm3d_kernels.hpp", "paper_2301_01868_amd/csrc/lbm3d_lattice.hpp",
                 "paper_2301_01868_amd/csrc/lbm3d_lib.hip", "paper_2301_01868_amd/build.py"]


def recorded_traffic(workload, prec_name, cells, kernel="k_step", sources=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    record (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when there is no record for this launch or the
    kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != step_source_hash(sources or STEP_SOURCES):
        return None
    e = rec.get("launches", {}).get(prec_name)
    if not e or e.get("cells") != cells:
        return None
    return int(e["hbm_bytes_per_launch"])


def workloads():
    from paper_2301_01868_amd import grids as G
    return {
        # the single-grid D2Q21 case: annulus R1 = 1, R2 = 2, 256 x 1024 uniform polar grid, tau 0.8
        "annulus_couette_256x1024": lambda: [G.workload_annulus_couette(256, 1024, tau=0.8)],
        # the seed-fixed 64-annulus ensemble (mixed D2Q9 / D2Q21), advanced as one batch
        "ensemble_64_annuli": lambda: G.workload_ensemble(),
        "planar_couette_q9_32x16": lambda: [G.workload_planar_couette_q9()],
        # kernel-scaling probe (not one of the stated workloads): the same annulus family at 16x the cells
        "annulus_couette_1024x4096": lambda: [G.workload_annulus_couette(1024, 4096, tau=0.8)],
        # one HBM-resident grid past 4 GiB per FP32 population buffer (5.6 GB): 67 M cells
        "annulus_couette_4096x16384": lambda: [G.workload_annulus_couette(4096, 16384, tau=0.8)],
        # general-mapping probe: a sheared, wobbled doubly periodic box whose metric terms depend on
        # q2, so the step rebuilds them per cell from the staged geometry
        "wobbled_box_q21_1024x1024": lambda: [G.periodic_box(21, 1024, 1024, dx=1.0, dy=1.1, skew=0.1, wobble=0.25,
                                                             tau=0.9)],
        # the wobbled box at HBM scale (8.4 M cells, 0.7 GB per FP32 population buffer)
        "wobbled_box_q21_2048x4096": lambda: [G.periodic_box(21, 2048, 4096, dx=1.0, dy=1.1, skew=0.1, wobble=0.25,
                                                             tau=0.9)],
        # the same box without the wobble: constant metric terms, so per-row tables (or, with
        # --geometry cell / cell_table, the per-cell paths on identical geometry)
        "sheared_box_q21_1024x1024": lambda: [G.periodic_box(21, 1024, 1024, dx=1.0, dy=1.1, skew=0.1, wobble=0.0,
                                                             tau=0.9)],
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _time_oracle(case, threads, target_s):
    import oracle
    o = oracle.OracleGrid(case)
    o.init(case.rho0)
    t0 = time.perf_counter()
    o.step(1, threads)
    per = max(time.perf_counter() - t0, 1e-6)
    k = max(1, min(200000, int(target_s / per)))
    t0 = time.perf_counter()
    o.step(k, threads)
    return k, time.perf_counter() - t0


def cpu_baseline(case, target_s=15.0, single_s=6.0):
    """Time the FP64 oracle (as it stands) on the host cores on a bounded
    sample of the workload: the same grid for as many steps as fit ~target_s
    with every core, then ~single_s on one core."""
    import oracle
    threads = oracle.max_threads()
    k, dt = _time_oracle(case, threads, target_s)
    k1, dt1 = _time_oracle(case, 1, single_s)
    return {"value": case.ncell * k / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%s: %d steps of the full %dx%d D2Q%d grid, FP64, %d OpenMP threads, %.1f s"
                      % (case.meta.get("workload", case.meta.get("problem", "grid")), k, case.n1, case.n2, case.q,
                         threads, dt),
            "single_core_value": case.ncell * k1 / dt1 / 1e6, "cpu_model": cpu_model()}


def measure(cases, prec, steps, warmup, wpb=0, stream=None, workload=None, unbatched=False, iterations=0, geometry=0):
    """Create, initialise and time `steps` steps of the workload; returns a dict.
    With unbatched=True a batched workload is also timed one grid at a time
    (each grid stepped alone through its own graphs, one after the other).
    iterations > 0 runs the fixed-point passes of the force relation instead
    of the lagged force."""
    import torch
    from paper_2301_01868_amd import lbm

    grids = []
    for c in cases:
        g = lbm.Grid(c, precision=prec, stream=ct_stream(stream), iterations=iterations, geometry=geometry)
        if wpb:
            g.set_launch(wpb)
        elif len(cases) == 1:
            # a single grid: enough steps per trial shape to time it above the noise
            # (about 4e8 lattice updates)
            g.autotune(max(10, min(200, int(4e8 // max(c.ncell, 1)))))
        else:
            g.autotune(10)
        g.init()
        grids.append(g)
    cells = sum(c.ncell for c in cases)
    batch = lbm.lbm_batch_create([g.h for g in grids]) if len(grids) > 1 else None
    if batch is not None:
        # each group's launch shape timed on the whole group (the per-grid choices above
        # serve the one-grid-at-a-time comparison); the trials advance every grid alike.
        # 64 launches per trial: with 20, two sessions with identical D2Q9 kernels kept
        # different shapes (169 against 178 us per launch)
        lbm.lbm_batch_autotune(batch, 64)

    def run(n):
        if batch is not None:
            lbm.lbm_batch_step(batch, n)
        else:
            grids[0].step(n)

    # a single grid captures its 32-step graph (per buffer parity) at its first
    # call of 32 steps or more: warm that up too, with an even count so the
    # timed steps start at the captured parity
    run(warmup if batch is not None else max(warmup, 32) + (max(warmup, 32) & 1))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    run(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    bads = [g.residual(check=False).bad_cells for g in grids]
    bad = sum(bads)
    unstable = [k for k, b in enumerate(bads) if b > 0]

    # dominant kernel: the D2Q21 step (algorithmic bytes 2 Q sizeof(population) per cell update)
    s_bytes = {lbm.LBM_FP64: 8, lbm.LBM_FP32: 4, lbm.LBM_FP16: 2}[prec]
    sname = {8: "f64", 4: "f32", 2: "f16"}[s_bytes]
    kind = {0: "row", 1: "cell tables", 2: "cell geometry"}[grids[0].info.table_kind]
    if batch is None:
        launch = (grids[0].info.waves_per_block, grids[0].info.waves_per_cu_cap)
        q = cases[0].q
        kcells = cells
        avg_ms = ms / steps
        kname = "k_step<%d,%s,%s>" % (q, sname, kind)
    else:
        groups = lbm.lbm_batch_groups(batch)
        gi = max(range(len(groups)), key=lambda k: (groups[k][0] == 21, groups[k][2]))
        q, _, kcells = groups[gi]
        reps = max(2, (steps // 4) // 2 * 2)
        lbm.lbm_batch_step_group(batch, gi, 2)
        torch.cuda.synchronize()
        ev0.record(stream)
        lbm.lbm_batch_step_group(batch, gi, reps)
        ev1.record(stream)
        torch.cuda.synchronize()
        avg_ms = ev0.elapsed_time(ev1) / reps
        kname = "k_step<%d,%s,%s> (batch group of %d cells)" % (q, sname, kind, kcells)
        launch = lbm.lbm_batch_group_launch(batch, gi)
    alg_bytes = 2 * q * s_bytes * kcells
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    traffic = recorded_traffic(workload, sname, kcells) if (workload and iterations == 0 and geometry == 0) else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
            "bytes_per_launch": alg_bytes, "avg_launch_us": round(avg_ms * 1e3, 3),
            "launch": {"waves_per_block": launch[0], "waves_per_cu_cap": launch[1]}}
    if traffic:
        roof["traffic_GBps"] = round(traffic / (avg_ms * 1e-3) / 1e9, 1)
    seq = None
    if batch is not None and unbatched:
        n1 = max(32, steps // 4)
        torch.cuda.synchronize()
        ev0.record(stream)
        for g in grids:
            g.step(n1)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms1 = ev0.elapsed_time(ev1)
        seq = {"value": round(cells * n1 / (ms1 * 1e-3) / 1e6, 1), "unit": "MLUPS",
               "ms_per_step": round(ms1 / n1, 5), "steps": n1}
    if batch is not None:
        lbm.lbm_batch_destroy(batch)
    for g in grids:
        g.close()
    return {"mlups": cells * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps, "cells": cells,
            "q21_cells": sum(c.ncell for c in cases if c.q == 21), "bad_cells": int(bad), "unstable": unstable,
            "roofline": roof, "unbatched": seq}


def measure3d(steps, warmup, stream):
    """The 3D step (39-velocity lattice, FP64) on a cylinder section continued
    along z: 128 radial x 512 azimuthal x 64 axial cells (4.19 M), radii 128 to
    256 lattice units, inner wall rotating at 0.05, tau 0.8; timed with HIP
    events on the grid's stream after warm-up steps."""
    import torch
    from paper_2301_01868_amd import grids3d as G3
    from paper_2301_01868_amd import lbm3d

    case = G3.circular_couette3(128, 512, 128.0, n3=64, dz=1.0, u_inner=0.05, tau=0.8)
    g = lbm3d.Grid3(case, stream=ct_stream(stream))
    g.init()
    # the step graph (32 steps per buffer parity) is captured in the warm-up
    g.step(max(warmup, 32) + (max(warmup, 32) & 1))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    g.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    m, U, Ut = g.moments()
    bad = int((~np.isfinite(m)).sum() + (m <= 0).sum())
    g.close()
    cells = case.ncell
    alg = 2 * 39 * 8 * cells          # one read and one write of every FP64 population
    achieved = alg / (ms / steps * 1e-3) / 1e9
    traffic = recorded_traffic("cylinder_couette_128x512x64", "f64", cells, kernel="k_step3", sources=STEP3_SOURCES)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "k_step3 (D3Q39, f64)", "bytes_per_launch": alg,
            "avg_launch_us": round(ms / steps * 1e3, 3)}
    if traffic:
        roof["traffic_GBps"] = round(traffic / (ms / steps * 1e-3) / 1e9, 1)
    return {"value": round(cells * steps / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(ms / steps, 5), "cells": cells, "bad_cells_after": bad,
            "workload": "cylinder_couette_128x512x64 (D3Q39, FP64)", "roofline": roof}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="ensemble_64_annuli", choices=sorted(workloads()))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--wpb", type=int, default=0)
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D (D3Q39, FP64) leg")
    ap.add_argument("--no-large", action="store_true", help="skip the single 4096 x 16384 grid leg")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark: continuous batching vs sequential FP64 on a Poisson trace")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="arrival rate (per s) for --serve; 0: offer --load of the measured capacity")
    ap.add_argument("--load", type=float, default=0.65)
    ap.add_argument("--requests", type=int, default=32, help="requests in the --serve trace")
    ap.add_argument("--cal-requests", type=int, default=48)
    ap.add_argument("--cal-seconds", type=float, default=20.0)
    ap.add_argument("--seq-sample", type=int, default=4, help="requests replayed sequentially in FP64")
    ap.add_argument("--fp64-above", type=float, default=None, metavar="STEPS",
                    help="serve requests whose slowest decay time exceeds STEPS with FP64 populations")
    ap.add_argument("--no-sequential", action="store_true",
                    help="serving: skip the sequential FP64 replay (long traces)")
    ap.add_argument("--geometry", default="auto", choices=["auto", "cell", "cell_table"],
                    help="metric terms per row when they allow it (auto), per cell rebuilt from the geometry in "
                         "the step (cell), or per cell from stored tables (cell_table)")
    ap.add_argument("--iterations", type=int, default=0,
                    help="fixed-point passes of the force relation (0: the paper's lagged force)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the library's plain copy kernel on MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one process drives one MI355X); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_01868_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        for _ in range(5):
            lbm.lbm_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, ct_stream(stream))
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        reps = 20
        ev0.record(stream)
        for _ in range(reps):
            lbm.lbm_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, ct_stream(stream))
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        with torch.cuda.stream(stream):
            ev0.record(stream)
            for _ in range(reps):
                dst.copy_(src)
            ev1.record(stream)
        torch.cuda.synchronize()
        ms_t = ev0.elapsed_time(ev1) / reps
        res = {"copy_probe_bytes": nbytes, "k_copy_GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
               "torch_copy_GBps": round(2 * nbytes / (ms_t * 1e-3) / 1e9, 1)}
        sink = torch.empty(8 << 20, dtype=torch.float32, device="cuda")
        for kind, name, mult in ((0, "nt_copy_GBps", 2), (1, "nt_read_GBps", 1), (2, "nt_write_GBps", 1)):
            d_ptr = sink.data_ptr() if kind == 1 else dst.data_ptr()
            lbm.lbm_bandwidth_probe(d_ptr, src.data_ptr(), nbytes, kind, ct_stream(stream))
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(reps):
                lbm.lbm_bandwidth_probe(d_ptr, src.data_ptr(), nbytes, kind, ct_stream(stream))
            ev1.record(stream)
            torch.cuda.synchronize()
            res[name] = round(mult * nbytes / (ev0.elapsed_time(ev1) / reps * 1e-3) / 1e9, 1)
        print(json.dumps(res), flush=True)
        return
    if args.serve:
        serve_bench(args)
        return
    cases = workloads()[args.workload]()
    stream = torch.cuda.Stream()
    it = args.iterations
    geom = {"auto": lbm.LBM_GEOM_AUTO, "cell": lbm.LBM_GEOM_CELL, "cell_table": lbm.LBM_GEOM_CELL_TABLE}[args.geometry]
    r32 = measure(cases, lbm.LBM_FP32, args.steps, args.warmup, args.wpb, stream, args.workload, unbatched=True,
                  iterations=it, geometry=geom)
    r64 = None
    if not args.no_fp64:
        r64 = measure(cases, lbm.LBM_FP64, max(2, args.steps // 2), max(2, args.warmup // 2), args.wpb, stream,
                      args.workload, iterations=it, geometry=geom)
    r16 = None
    if not args.no_fp16:
        r16 = measure(cases, lbm.LBM_FP16, args.steps, args.warmup, args.wpb, stream, args.workload, iterations=it,
                      geometry=geom)

    rl = None
    if not args.no_large and it == 0 and geom == lbm.LBM_GEOM_AUTO:
        big = "annulus_couette_4096x16384"
        rl = measure(workloads()[big](), lbm.LBM_FP32, max(8, args.steps // 10), max(2, args.warmup // 10), args.wpb,
                     stream, big)
        rl = {"workload": big, "value": round(rl["mlups"], 1), "unit": "MLUPS",
              "ms_per_step": round(rl["ms_per_step"], 5), "cells": rl["cells"], "roofline": rl["roofline"],
              "bad_cells_after": rl["bad_cells"]}

    r3 = None
    if not args.no_3d and it == 0 and geom == lbm.LBM_GEOM_AUTO:
        r3 = measure3d(max(4, args.steps // 2), max(2, args.warmup // 2), stream)

    cpu = None
    if not args.no_cpu:
        q21 = sorted([c for c in cases if c.q == 21] or cases, key=lambda c: c.ncell)
        cpu = cpu_baseline(q21[len(q21) // 2])    # the median-sized D2Q21 grid of the workload

    out = {
        "metric": "MLUPS + % HBM roofline (D2Q21 FP32 vs FP64)",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": r32["cells"], "q21_cells": r32["q21_cells"],
                   "grids": len(cases), "precision": "fp32 populations (offsets from the local rest state)",
                   "force": "lagged" if it == 0 else "%d fixed-point passes" % it, "geometry": args.geometry,
                   "bad_cells_after": r32["bad_cells"], "unstable_instances": r32["unstable"]},
        "roofline": r32["roofline"],
        "cpu_baseline": cpu,
    }
    if r32["unbatched"] is not None:
        out["unbatched_fp32"] = r32["unbatched"]
    if r64 is not None:
        out["fp64"] = {"value": round(r64["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64["ms_per_step"], 5),
                       "roofline": r64["roofline"], "bad_cells_after": r64["bad_cells"]}
    if r16 is not None:
        out["fp16"] = {"value": round(r16["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r16["ms_per_step"], 5),
                       "roofline": r16["roofline"], "bad_cells_after": r16["bad_cells"]}
    if rl is not None:
        out["single_grid_fp32"] = rl
    if r3 is not None:
        out["d3q39_fp64"] = r3
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """Serving: Poisson arrivals of steady-state solves drawn from the planar
    and circular Couette / Poiseuille families (wall-normal N log-uniform over
    16..512, N x 4N cells, tau in 0.55..1, D2Q9 or D2Q21), continuous
    batching in FP32 to residual 1e-8 under an 8 GB budget, against plain
    sequential FP64 stepping on a seeded sample of the same requests.

    The stated 50 requests/s offers far more work than one GPU can do (the
    mean request needs about 1e11 lattice updates), so the batched capacity
    is measured first (a burst of requests from the same distribution, all
    present at the start) and the arrival rate is set to offer `--load` of it;
    the stated rate's offered load is reported beside it."""
    import copy
    import torch
    from paper_2301_01868_amd import serve, lbm

    def note(text):
        print(text, file=sys.stderr, flush=True)

    stream, setup = torch.cuda.Stream(), torch.cuda.Stream()
    budget = 8 << 30
    tol = 1e-8
    mean_lu = serve.mean_predicted_lu(n_min=16, n_max=512, tol=tol)
    # 1. batched capacity on this request mix
    cal = serve.make_trace(seed=2301_01870, rate=1e9, n_requests=args.cal_requests, tol=tol)
    srv = serve.Server(hbm_budget=budget, check_every=256, stream=stream, setup_stream=setup,
                       fp64_above=args.fp64_above)
    note("capacity run: %d requests for %.0f s" % (len(cal), args.cal_seconds))
    st = srv.run(cal, realtime=False, stop_after=args.cal_seconds, progress=note)
    capacity = st["lattice_updates"] / st["makespan"]
    note("capacity %.3g lattice updates/s" % capacity)
    # 2. the served trace
    rate = args.rate if args.rate > 0 else args.load * capacity / mean_lu
    trace = serve.make_trace(seed=2301_01869, rate=rate, n_requests=args.requests, tol=tol)
    base = copy.deepcopy(trace)
    srv = serve.Server(hbm_budget=budget, check_every=256, stream=stream, setup_stream=setup,
                       fp64_above=args.fp64_above)
    note("served trace: %d requests at %.4g per s" % (len(trace), rate))
    info = srv.run(trace, realtime=True, progress=note)
    s_b = serve.summarize(trace, info["makespan"])
    s_b.update({k: info[k] for k in ("rounds", "setup_s", "check_s", "retire_s", "peak_resident")})
    # 3. sequential FP64 on a seeded sample, back to back (service times only)
    seq = None
    diffs = []
    if not args.no_sequential and args.seq_sample > 0:
        rng = np.random.default_rng(11)
        idx = sorted(rng.choice(len(base), min(args.seq_sample, len(base)), replace=False).tolist())
        sample = [base[i] for i in idx]
        for r in sample:
            r.arrival = 0.0
        note("sequential FP64 replay of requests %s" % idx)
        info2 = serve.run_sequential(sample, precision=lbm.LBM_FP64, check_every=256, stream=ct_stream(stream),
                                     realtime=False, progress=note)
        lu_s = sum(r.steps * r.case.ncell for r in sample)
        ok = [r for r in sample if r.status == "converged"]
        seq = {"sample": idx, "requests": len(sample), "converged": len(ok),
               "solves_per_s": len(ok) / info2["makespan"], "lattice_updates": lu_s,
               "lu_per_s": lu_s / info2["makespan"], "makespan_s": info2["makespan"],
               "service_s": [round(r.finish - r.start, 3) for r in sample],
               "statuses": [r.status for r in sample], "steps": [r.steps for r in sample]}
        # equal accuracy: both converged to the residual; velocities against the speed scale 0.05
        for i, b in zip(idx, sample):
            a = trace[i]
            if a.status == "converged" and b.status == "converged":
                diffs.append({"rid": i, "family": a.case.meta["draw"]["family"], "N": a.case.n1, "q": a.case.q,
                              "tau": round(a.case.tau, 4), "served_precision": {0: "fp64", 1: "fp32", 2: "fp16"}.get(
                                  a.precision, a.precision), "slowest_decay_steps": round(serve.slow_decay_steps(a.case)),
                              "steps_served": a.steps, "steps_fp64": b.steps,
                              "max_diff_u_over_U": float(np.abs(a.result["u"] - b.result["u"]).max() / 0.05)})
    out = {"metric": "solves/s, p50/p99 latency (serving)", "value": round(s_b["solves_per_s"], 4),
           "unit": "solves/s", "higher_is_better": True, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "poisson_trace_config5", "requests": len(trace), "rate_per_s": rate,
                      "n_wall_normal": "log-uniform 16..512, N x 4N cells", "tol": tol, "hbm_budget_bytes": budget,
                      "check_every": 256, "fp64_above_decay_steps": args.fp64_above,
                      "fp64_requests": sum(r.precision == lbm.LBM_FP64 for r in trace)},
           "offered_load": {"mean_predicted_lu_per_request": mean_lu, "offered_lu_per_s": rate * mean_lu,
                            "capacity_lu_per_s": capacity, "load_fraction": rate * mean_lu / capacity,
                            "stated_rate_per_s": 50.0, "stated_offered_lu_per_s": 50.0 * mean_lu,
                            "stated_over_capacity": 50.0 * mean_lu / capacity,
                            "capacity_run": {"requests": len(cal), "seconds": st["makespan"],
                                             "lattice_updates": st["lattice_updates"],
                                             "peak_resident": st["peak_resident"]}},
           "batched_fp32": s_b, "sequential_fp64": seq,
           "capacity_over_sequential_lu_per_s": (capacity / seq["lu_per_s"]) if seq else None,
           "served_vs_fp64": {"max_diff_u_over_U": max(d["max_diff_u_over_U"] for d in diffs) if diffs else None,
                            "requests": diffs}}
    print(json.dumps(out), flush=True)


def ct_stream(torch_stream):
    import ctypes
    return ctypes.c_void_p(torch_stream.cuda_stream) if torch_stream is not None else None


if __name__ == "__main__":
    main()
