"""Throughput benchmark of the curvilinear lattice Boltzmann step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precision fp32|fp64]

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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def workloads():
    from paper_2301_01868_amd import grids as G
    return {
        # the single-grid D2Q21 case: annulus R1 = 1, R2 = 2, 256 x 1024 uniform polar grid, tau 0.8
        "annulus_couette_256x1024": lambda: [G.workload_annulus_couette(256, 1024, tau=0.8)],
        # the seed-fixed 64-annulus ensemble (mixed D2Q9 / D2Q21), advanced as one batch
        "ensemble_64_annuli": lambda: G.workload_ensemble(),
        "planar_couette_q9_32x16": lambda: [G.workload_planar_couette_q9()],
    }


def cpu_baseline(case, target_s=15.0):
    """Time the FP64 oracle (as it stands) on the host cores on a bounded
    sample of the workload: the same grid for as many steps as fit ~target_s."""
    import oracle
    o = oracle.OracleGrid(case)
    o.init(case.rho0)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    o.step(1, threads)
    t1 = time.perf_counter()
    per = max(t1 - t0, 1e-6)
    k = max(1, min(2000, int(target_s / per)))
    t0 = time.perf_counter()
    o.step(k, threads)
    dt = time.perf_counter() - t0
    lups = case.ncell * k / dt
    return {"value": lups / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%s, %d steps of the full %dx%d grid, FP64, %d OpenMP threads, %.1f s"
                      % (case.meta.get("workload", "grid"), k, case.n1, case.n2, threads, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="annulus_couette_256x1024", choices=sorted(workloads()))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--wpb", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each box has one MI355X); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2301_01868_amd import lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prec = lbm.LBM_FP32 if args.precision == "fp32" else lbm.LBM_FP64
    cases = workloads()[args.workload]()
    stream = torch.cuda.Stream()
    grids = []
    for c in cases:
        g = lbm.Grid(c, precision=prec, stream=ct_stream(stream))
        if args.wpb:
            g.set_launch(args.wpb)
        g.init()
        grids.append(g)
    cells = sum(c.ncell for c in cases)
    batch = lbm.lbm_batch_create([g.h for g in grids]) if len(grids) > 1 else None

    def run(n):
        if batch is not None:
            lbm.lbm_batch_step(batch, n)
        else:
            grids[0].step(n)

    run(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    run(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / args.steps
    mlups = cells * args.steps / (ms * 1e-3) / 1e6

    # roofline of the dominant kernel: the D2Q21 step (algorithmic bytes 2 Q s per cell update)
    s_bytes = 4 if prec == lbm.LBM_FP32 else 8
    q21_cells = sum(c.ncell for c in cases if c.q == 21)
    q9_cells = cells - q21_cells
    if batch is None:
        dom_q = cases[0].q
        alg_bytes = 2 * dom_q * s_bytes * cells
        avg_launch_ms = ms_step
    else:
        # time the batch with only its D2Q21 group launched, same stream, events
        dom_q = 21
        alg_bytes = 2 * 21 * s_bytes * q21_cells
        avg_launch_ms = None
    roof = None
    if avg_launch_ms:
        achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_step<%d,%s>" % (dom_q, args.precision), "bytes_per_launch": alg_bytes,
                "avg_launch_us": round(avg_launch_ms * 1e3, 3)}

    # residual sanity (finite state) after the timed steps
    bad = 0
    for g in grids:
        r = g.residual(check=False)
        bad += r.bad_cells

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cases[0] if len(cases) == 1 else max((c for c in cases if c.q == 21), key=lambda c: -c.ncell))

    out = {
        "metric": "MLUPS + % HBM roofline (D2Q21 FP32 vs FP64)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == lbm.LBM_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": cells, "q21_cells": q21_cells, "q9_cells": q9_cells,
                   "grids": len(cases), "precision": args.precision, "bad_cells_after": int(bad)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if batch is not None:
        lbm.lbm_batch_destroy(batch)


def ct_stream(torch_stream):
    import ctypes
    return ctypes.c_void_p(torch_stream.cuda_stream)


if __name__ == "__main__":
    main()
