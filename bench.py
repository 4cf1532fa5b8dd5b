#!/usr/bin/env python3
"""Throughput of the explicit FV Euler hot path on one MI355X.

One step = one full SSP-RK3 step (3 stage kernels: ghost resolve + MUSCL +
Roe + flux divergence + stage update, then the step-end reductions) over the
whole grid.  The headline workload is the 2D supersonic-inlet-like
multi-block grid (4 blocks of 512 x 256 cells, sheared wavy curvilinear mesh,
Mach 4 inflow of the paper's inflow table, slip walls, extrapolation outflow)
in FP64.  Inputs are synthetic and already resident in HBM when the timed
region starts.

Printed: one JSON line with cell-updates/s, the roofline of the stage kernel
(algorithmic bytes per launch / average launch time from HIP events) and the
CPU reference timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s + % HBM roofline; batched p50/p99 solve latency vs plain"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_cell_step(case) -> int:
    """Compulsory HBM bytes of one SSP-RK3 step per cell (FP64 state).

    stage 1 reads U^n and writes U1; stages 2 and 3 read their stage state and
    U^n and write the next state: 8 state-sized transfers of nv doubles.
    Curvilinear 2D grids also read the node coordinates in every stage
    (2 doubles per cell).  Reductions are fused and ghost cells are never
    stored, so they add nothing."""
    nv = case.nv
    b = 8 * 8 * nv
    if any(blk.x is not None for blk in case.blocks):
        b += 3 * 16
    return b


def time_grid(fv, case, params, steps, warmup):
    import torch
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    if warmup:
        g.step(params, warmup)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    info = g.step(params, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = e0.elapsed_time(e1)
    # per-kernel timing pass over the same number of steps
    _, stage_ms = g.step_timed(params, steps)
    st = g.stats()
    return g, info, wall, dev_ms, stage_ms, st


def roofline_of(case, stage_ms, steps):
    cells = case.ncells
    per_step = algorithmic_bytes_per_cell_step(case) * cells
    launches = 3 * steps
    avg_ms = float(sum(stage_ms[:3])) / launches
    bytes_per_launch = per_step / 3.0
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                kernel="k_stage2d" if case.ndim == 2 else "k_stage3d",
                bytes_per_launch=int(bytes_per_launch), avg_launch_ms=round(avg_ms, 5),
                finalize_avg_ms=round(float(stage_ms[3]) / steps, 5))


def cpu_baseline(case, budget_s=12.0):
    from oracle import oracle as O
    ref = O.OracleGrid(case)
    t0 = time.perf_counter()
    ref.run(case.params, 1)
    t1 = time.perf_counter() - t0
    n = max(1, min(200, int(budget_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    ref.run(case.params, n)
    dt = time.perf_counter() - t0
    return dict(value=round(case.ncells * n / dt, 1), unit="cell-updates/s",
                cores=O.num_threads(), kind="oracle",
                sample=f"{case.name}: {n} SSP-RK3 steps of the full {case.ncells}-cell grid "
                       f"({dt:.1f} s wall, FP64, OpenMP over faces/cells)")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE={world}) is not "
              "supported: the hot path is measured on a single MI355X and would shard by "
              "blocks / instances across GPUs (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_18057_amd import cases, fv
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fv.lib()

    # ---- headline: 2D inlet-like 4 x 512 x 256, FP64
    case = cases.inlet_2d()
    prm = case.params
    log(f"[bench] headline {case.name} cells={case.ncells} steps={args.steps} warmup={args.warmup}")
    g, info, wall, dev_ms, stage_ms, st = time_grid(fv, case, prm, args.steps, args.warmup)
    ms_per_step = dev_ms / args.steps
    value = case.ncells * args.steps / (dev_ms * 1e-3)
    roof = roofline_of(case, stage_ms, args.steps)
    log(f"[bench] {value/1e9:.3f} G cell-updates/s, {ms_per_step*1e3:.1f} us/step, "
        f"stage kernel {roof['avg_launch_ms']*1e3:.1f} us -> {roof['achieved']:.0f} GB/s")
    del g

    extra = {}
    if not args.no_extra:
        for name, mk, prec, steps in [
            ("inlet_2d_fp32flux", cases.inlet_2d, cases.FP32_FLUX, args.steps),
            ("blobs_3d_fp64", cases.blobs_3d, cases.FP64, 50),
            ("blobs_3d_fp32flux", cases.blobs_3d, cases.FP32_FLUX, 50),
        ]:
            c = mk()
            p = cases.Params(**{**c.params.__dict__, "precision": prec})
            log(f"[bench] extra {name} cells={c.ncells} steps={steps}")
            gx, ix, wx, dx, sx, stx = time_grid(fv, c, p, steps, 5)
            rx = roofline_of(c, sx, steps)
            extra[name] = dict(value=round(c.ncells * steps / (dx * 1e-3), 1),
                               ms_per_step=round(dx / steps, 5), roofline=rx,
                               tile=dict(rows=stx["tile_rows"], ny=stx["tile_ny"],
                                         tiles=stx["tiles"], blocks=stx["launch_blocks"]))
            log(f"[bench]   {extra[name]['value']/1e9:.3f} G cell-updates/s, "
                f"{rx['achieved']:.0f} GB/s ({100*rx['frac']:.1f}% HBM)")
            del gx

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU reference on a bounded sample")
        cpu = cpu_baseline(case)
        log(f"[bench] cpu {cpu['value']/1e6:.2f} M cell-updates/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "inlet_2d: 2D Euler, 4 blocks x 512x256 cells on the sheared wavy "
                        "inlet-like curvilinear mesh, Mach 4 inflow (p=12270 Pa, T=217 K), "
                        "slip walls, extrapolation outflow, MUSCL-minmod + Roe, SSP-RK3, CFL 0.5",
            "cells": case.ncells,
            "precision": "fp64",
            "tile_rows": st["tile_rows"],
            "tiles": st["tiles"],
            "launch_blocks": st["launch_blocks"],
            "parallelism": "single GPU",
        },
        "ssspnt": round(1e-6 * case.ncells * 3 * args.steps / (dev_ms * 1e-3), 2),
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
