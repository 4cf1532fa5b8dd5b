#!/usr/bin/env python3
"""Throughput of the explicit FV Euler hot path on one MI355X.

One step = one full SSP-RK3 step (3 stage kernels: ghost resolve + MUSCL +
Roe + flux divergence + stage update, then the step-end reductions) over the
whole grid.  The headline workload is the 2D supersonic-inlet-like
multi-block grid (4 blocks of 512 x 256 cells, sheared wavy curvilinear mesh,
Mach 4 inflow of the paper's inflow table, slip walls, extrapolation outflow)
in FP64.  Inputs are synthetic and already resident in HBM when the timed
region starts; tile shapes come from the autotuner before timing.

Printed: one JSON line with cell-updates/s, the roofline of the stage kernel
(algorithmic bytes per launch / average launch time from HIP events on the
launch stream), the CPU reference timed on a bounded sample on this host,
and (unless --no-extra) the FP32-flux and 3D workloads, the 64-instance
batch and the serving trace.

``--summarize DIR`` turns rocprofv3 CSV output (kernel trace stats or
counter collection) into the short text summaries kept under profiles/.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RAMP_S = 0.25          # untimed load before each timed run (clock ramp)
FP64_PEAK_TFS = 78.6   # vector FP64, 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_TFS = 157.3
METRIC = "cell-updates/s + % HBM roofline; batched p50/p99 solve latency vs plain"
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2305_18057_amd", "csrc")


def _cases():
    from paper_2305_18057_amd import cases
    return cases


# workload makers by name
WORKLOADS = {
    "inlet_2d": lambda: _cases().inlet_2d(),
    "blobs_3d": lambda: _cases().blobs_3d(),
    "inlet_2d_ns": lambda: _cases().inlet_2d_ns(),
    "curv3d_mms": lambda: _cases().curv3d_mms(192),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# algorithmic figures per cell
# --------------------------------------------------------------------------
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
        # node coordinates, read in every stage: about one node per cell
        b += 3 * (24 if case.ndim == 3 else 16)
    if getattr(case, "source", None) is not None:
        b += 3 * 8 * nv  # the source S_h, read in every stage
    return b


def algorithmic_flops_per_cell_stage(case) -> int:
    """FP64 operations of one cell-stage counted from the formulas (add, mul,
    div, sqrt, abs/min/max each 1; a fused multiply-add 2), averaged over the
    three stages: ND face fluxes (each face flux is formed once and used by
    the two cells it separates), the reconstruction of every variable in every
    direction, the flux divergence, the stage update and the fused norm / CFL
    reductions.  Newton steps of reciprocals and roots are not counted."""
    nd = case.ndim
    curv = any(blk.x is not None for blk in case.blocks)
    if nd == 2:
        flux = 140 + (7 if curv else -6)  # general normal (+ |S|, n) or axis-aligned
        recon = 5 * 4 * 2
        div = 3 * 4
        upd = 17 + (11 if curv else 0)    # + volume and face vectors from nodes
        red = 19
        return 2 * flux + recon + div + upd + red
    curv = any(getattr(blk, "z", None) is not None for blk in case.blocks)
    flux = 155 + (12 if curv else 0)  # + |S| and n of a general normal
    recon = 5 * 5 * 3
    div = 5 * 5
    upd = 21
    red = 19
    # curvilinear: three face vectors per cell (each shared by two cells):
    # diagonals 6, cross product 9 + halving 3, centre 12, S . centre 5; the
    # volume from the six S . centre values 7.  Source: - |Omega| S_h, 10.
    metrics = (3 * 35 + 7) if curv else 0
    src = 10 if getattr(case, "source", None) is not None else 0
    return 3 * flux + recon + div + upd + red + metrics + src


# --------------------------------------------------------------------------
# committed profile summaries (traffic and instruction counts)
# --------------------------------------------------------------------------
def is_viscous(case) -> bool:
    """The case runs the Navier-Stokes stage kernel (viscosity or no-slip wall)."""
    return getattr(case.params, "mu", 0.0) > 0.0 or any(
        bc.kind == 5 for blk in case.blocks for bc in blk.bc)


def is_general3d(case) -> bool:
    """The case runs the general 3D stage kernel (curvilinear blocks or a source)."""
    return case.ndim == 3 and (getattr(case, "source", None) is not None or any(
        getattr(blk, "z", None) is not None for blk in case.blocks))


def stage_kernel(case) -> str:
    if case.ndim == 3:
        return "k_stage3d_gen" if is_general3d(case) else "k_stage3d"
    return "k_stage2d_ns" if is_viscous(case) or getattr(case, "source", None) is not None \
        else "k_stage2d"


def kernel_sources_sha(ndim: int, ns: bool = False, gen: bool = False) -> str:
    h = hashlib.sha256()
    if ndim == 3:
        src = "fv_kernels3d_gen.hip" if gen else "fv_kernels3d.hip"
    else:
        src = "fv_kernels2d_ns.hip" if ns else "fv_kernels2d.hip"
    for f in ("fv_device.h", src):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(kernel: str, workload: str, ndim: int):
    """key: value lines of profiles/<kernel>_<workload>_counters.txt, or None
    when absent or taken from kernel sources other than the current ones."""
    ns = kernel.endswith("_ns")
    gen = kernel.endswith("_gen")
    path = os.path.join(PROFILES, f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_sources_sha") != kernel_sources_sha(ndim, ns, gen):
        return None
    return rec


# --------------------------------------------------------------------------
# single-grid timing
# --------------------------------------------------------------------------
def ramp_clocks(g, params, U0, seconds=RAMP_S):
    """Untimed steps for `seconds`, then the initial state back: the GPU's
    clocks rise over tens of milliseconds of load, and a short timed window
    started from idle would measure the ramp rather than the solver."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        g.step(params, 50)
    torch.cuda.synchronize()
    g.set_state(U0)


def time_grid(fv, case, params, steps, warmup, tune_cache=None, stage_times=True):
    import torch
    g = fv.Grid(case)
    U0 = case.state_flat()
    g.set_state(U0)
    if tune_cache is not None:
        g.tune(params, tune_cache)
        g.set_state(U0)
    ramp_clocks(g, params, U0)
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
    # per-kernel timing pass over the same number of steps (HIP events around
    # every stage launch on the grid's stream; SSP-RK3 only)
    stage_ms = g.step_timed(params, steps)[1] if stage_times else None
    st = g.stats()
    return g, info, wall, dev_ms, stage_ms, st


def repeat_timing(fv, case, params, steps, reps=5, tune_cache=None):
    """Median of `reps` timed runs of `steps` steps, each from the initial
    state restored from a device copy (clock ramp and 5 warm-up steps
    first)."""
    import torch
    g = fv.Grid(case)
    U0 = torch.from_numpy(case.state_flat()).to("cuda")
    g.set_state(U0)
    if tune_cache is not None:
        g.tune(params, tune_cache)
        g.set_state(U0)
    ramp_clocks(g, params, U0)
    g.step(params, 5)
    stream = torch.cuda.current_stream()
    per = []
    for _ in range(reps):
        g.set_state(U0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step(params, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / steps)
    g.close()
    med = float(np.median(per))
    return dict(reps=reps, steps=steps, ms_per_step=[round(x, 5) for x in per],
                median_ms_per_step=round(med, 5),
                median_cell_updates_per_s=round(case.ncells / (med * 1e-3), 1))


def copy_bandwidth():
    """Achievable device bandwidth: best of 5 timed 1 GiB device-to-device
    copies, counting the bytes read and written."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return round(2 * n * 8 / (best * 1e-3) / 1e9, 1)


def bench_rk_schemes(fv, cases, tune_cache, steps2d):
    """The paper's 2- and 4-stage second-order schemes beside SSP-RK3 on the
    2D inlet and 3D blobs grids (FP64): per-step time, cell-updates/s and
    ssspnt with the substeps counted (Sec. 7, Eq. ssspnt), the measure by
    which the paper compares its RK2 and RK4 runs."""
    out = {}
    for wl, mk, steps in (("inlet_2d", cases.inlet_2d, steps2d), ("blobs_3d", cases.blobs_3d, 20)):
        c = mk()
        rows = {}
        for rk, nst in ((2, 2), (3, 3), (4, 4)):
            p = cases.Params(**{**c.params.__dict__, "precision": cases.FP64, "rk": rk})
            gx, ix, wx, dx, _, stx = time_grid(fv, c, p, steps, 5, tune_cache, stage_times=False)
            rows[f"rk{rk}"] = dict(stages=nst, ms_per_step=round(dx / steps, 5),
                                   cell_updates_per_s=round(c.ncells * steps / (dx * 1e-3), 1),
                                   ssspnt=round(1e-6 * c.ncells * nst * steps / (dx * 1e-3), 2))
            gx.close()
            del gx
        base = rows["rk3"]["ssspnt"]
        for r in rows.values():
            r["ssspnt_vs_rk3"] = round(r["ssspnt"] / base, 4)
        out[wl] = dict(cells=c.ncells, steps=steps, **rows)
        log(f"[bench] rk schemes {wl}: " + ", ".join(
            f"{k} {v['ms_per_step']*1e3:.1f} us/step ssspnt {v['ssspnt']:.0f}" for k, v in rows.items()))
    return out


def bench_hetero(fv, cases, tune_cache, steps=20, workers=16, viscous=False):
    """The CPU-GPU heterogeneous mode (Sec. 4 workflow, Sec. 6 model) on the
    inlet-like grid as one 2048 x 256 block, FP64, with the Euler solver or
    (viscous) the Navier-Stokes solver of the viscous inlet workload (no-slip
    walls, mu = 1.5e-2; Sec. 8 measures both): the pure-GPU step time, one
    host core's time per cell, a sweep of the workload ratio r (the cells
    of the GPU over the cells of one of `workers` host workers) with the
    measured time per step, and the model of Sec. 6 fitted to the sweep:
    t_I is the rate of one worker among `workers` (the slope of the host
    part's time over its cells per worker), r_gc the pure GPU's speed over
    that, kappa = (1 + alpha) beta by least squares; alpha quoted for the
    paper's beta range 0.2 .. 0.5.  With the Navier-Stokes solver also the
    influence of the problem size (Sec. 8): the ratio sweep on a quarter
    and on twice the cells."""
    from paper_2305_18057_amd import perfmodel as PM

    def setup(Nl, Nw):
        c = cases.inlet_case(Nl, Nw, 1, name=("inlet_2d_ns_1block" if viscous else "inlet_2d_1block"))
        if viscous:
            for f in (2, 3):
                c.blocks[0].bc[f] = cases.BC(cases.NOSLIP)
            c.params = cases.Params(**{**c.params.__dict__, "mu": 1.5e-2, "prandtl": 0.72})
        p = cases.Params(**{**c.params.__dict__, "precision": cases.FP64})
        gx, _, _, dx, _, _ = time_grid(fv, c, p, steps, 5, tune_cache, stage_times=False)
        gx.close()
        return c, p, dx / steps * 1e-3

    def runner(c, p):
        U0 = c.state_flat()

        def run(split, nw, n=steps):
            h = fv.Hetero(c, split, nw)
            h.set_state(U0)
            h.step(p, 3)
            h.set_state(U0)
            info = h.step(p, n)
            h.close()
            return [t / n * 1e-3 for t in info["times_ms"]]
        return run

    Nl, Nw = 2048, 256
    c, p, t_gpu = setup(Nl, Nw)
    N = c.ncells
    run = runner(c, p)

    # one host core: its time per cell-step from the host part's substep time
    # of 16 columns (context; the model takes the workers' own rate, below)
    one = run(Nl - 16, 1)
    tI_core = one[1] / (16 * Nw)
    rows = []
    for nc in (2, 4, 8, 16, 32, 64, 128):
        split = Nl - nc
        r = split * workers / nc
        tm = run(split, workers)
        rows.append(dict(cpu_columns=nc, ratio=round(r, 1), wall_ms=round(tm[3] * 1e3, 4),
                         gpu_ms=round(tm[0] * 1e3, 4), host_ms=round(tm[1] * 1e3, 4),
                         exchange_ms=round(tm[2] * 1e3, 4),
                         ssspnt=round(1e-6 * N * 3 / tm[3], 2)))
    # t_I of one of the `workers` running together: the slope of the host
    # part's time per step over its cells per worker (the intercept is the
    # pool's own per-step cost).  The model's C workers each take t_I per
    # cell, so the rate they reach together on this host is the one to use.
    tI, host_fixed = PM.worker_tI([x["cpu_columns"] * Nw / workers for x in rows],
                                  [x["host_ms"] * 1e-3 for x in rows])
    r_gc = N * tI / t_gpu
    fit = PM.fit_kappa(Nl, Nw, 1, workers, [x["ratio"] for x in rows],
                       [x["wall_ms"] * 1e-3 for x in rows], r_gc, tI)
    for x in rows:
        x["model_ms"] = round(PM.time_ratio(Nl, Nw, 1, workers, x["ratio"], r_gc, tI, fit.kappa) * 1e3, 4)
    best = min(rows, key=lambda x: x["wall_ms"])
    out = dict(solver="navier-stokes" if viscous else "euler", cells=N, steps=steps,
               workers=workers, pure_gpu_ms=round(t_gpu * 1e3, 4),
               pure_gpu_ssspnt=round(1e-6 * N * 3 / t_gpu, 2),
               host_core_tI_ns=round(tI_core * 1e9, 2),
               host_core_cell_updates_per_s=round(1 / tI_core, 1),
               host_worker_tI_ns=round(tI * 1e9, 2), host_pool_fixed_ms=round(host_fixed * 1e3, 4),
               r_gc=round(r_gc, 1), kappa=round(fit.kappa, 3), fit_rms_rel=round(fit.rms_rel, 4),
               alpha_at_beta_0_2=round(fit.alpha(0.2), 2), alpha_at_beta_0_5=round(fit.alpha(0.5), 2),
               model_balance_ms=round(PM.time_ratio(Nl, Nw, 1, workers, r_gc, r_gc, tI, fit.kappa) * 1e3, 4),
               best=dict(ratio=best["ratio"], wall_ms=best["wall_ms"],
                         vs_pure_gpu=round(t_gpu * 1e3 / best["wall_ms"], 4)),
               sweep=rows)
    if viscous:
        # the influence of the problem size: the same sweep on a quarter and
        # on twice the cells (host columns scaled with N_l; finer along i
        # only: refined across the no-slip walls, the impulsive Mach 4 start
        # turns non-physical)
        sizes = []
        for sl, sw in ((1024, 128), (4096, 256)):
            cs, ps, tg = setup(sl, sw)
            rs = runner(cs, ps)
            pts = []
            for ncs in sorted({max(2, nc * sl // Nl) for nc in (2, 4, 8, 16, 32, 64, 128)}):
                tm = rs(sl - ncs, workers)
                pts.append(dict(cpu_columns=ncs, ratio=round((sl - ncs) * workers / ncs, 1),
                                wall_ms=round(tm[3] * 1e3, 4),
                                ssspnt=round(1e-6 * cs.ncells * 3 / tm[3], 2)))
            b = min(pts, key=lambda x: x["wall_ms"])
            sizes.append(dict(cells=cs.ncells, shape=[sl, sw], pure_gpu_ms=round(tg * 1e3, 4),
                              pure_gpu_ssspnt=round(1e-6 * cs.ncells * 3 / tg, 2),
                              best=dict(ratio=b["ratio"], wall_ms=b["wall_ms"],
                                        vs_pure_gpu=round(tg * 1e3 / b["wall_ms"], 4)),
                              sweep=pts))
            log(f"[bench] hetero navier-stokes {sl} x {sw}: pure GPU {tg * 1e3:.4f} ms/step, best "
                f"ratio {b['ratio']} at {b['wall_ms']} ms/step ({tg * 1e3 / b['wall_ms']:.3f}x)")
        out["problem_sizes"] = sizes
    log(f"[bench] hetero {out['solver']}: pure GPU {out['pure_gpu_ms']} ms/step, host core "
        f"{1e-6 / tI_core:.2f} M cell-updates/s, worker t_I {tI * 1e9:.0f} ns, "
        f"r_gc {r_gc:.0f}; best ratio {best['ratio']} at {best['wall_ms']} ms/step "
        f"({out['best']['vs_pure_gpu']}x pure GPU); kappa {fit.kappa:.2f} (fit rms {fit.rms_rel:.2f})")
    return out


def roofline_of(case, stage_ms, steps, workload, fp32=False):
    cells = case.ncells
    kernel = stage_kernel(case)
    per_step = algorithmic_bytes_per_cell_step(case) * cells
    launches = 3 * steps
    avg_ms = float(sum(stage_ms[:3])) / launches
    bytes_per_launch = per_step / 3.0
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    rec = profile_record(kernel, workload + ("_fp32flux" if fp32 else "_fp64"), case.ndim)
    traffic = None
    if rec is not None and "hbm_bytes_per_launch" in rec:
        traffic = int(float(rec["hbm_bytes_per_launch"]))
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                kernel=kernel, bytes_per_cell_step=algorithmic_bytes_per_cell_step(case),
                bytes_per_launch=int(bytes_per_launch), avg_launch_ms=round(avg_ms, 5),
                finalize_avg_ms=round(float(stage_ms[3]) / steps, 5))
    if rec is not None and "trace_avg_us_per_launch" in rec:
        # the profile's execution time per launch, beside the event time above
        # (which also holds each launch's dispatch and completion)
        tr = float(rec["trace_avg_us_per_launch"]) * 1e-3
        roof["trace_avg_launch_ms"] = round(tr, 5)
        roof["trace_achieved"] = round(bytes_per_launch / (tr * 1e-3) / 1e9, 1)
    if is_viscous(case):
        # the flop count above is the inviscid one; the viscous kernel reports
        # its measured instruction figures only
        alu = dict(peak_tflops=FP32_PEAK_TFS if fp32 else FP64_PEAK_TFS)
        if rec is not None:
            for k in ("valu_instr_per_cell_stage", "valu_busy_frac", "wait_frac", "vgprs",
                      "scratch_bytes_per_lane"):
                if k in rec:
                    alu[k] = float(rec[k])
        return roof, alu
    flops = algorithmic_flops_per_cell_stage(case)
    tfs = flops * cells / (avg_ms * 1e-3) / 1e12
    peak = FP32_PEAK_TFS if fp32 else FP64_PEAK_TFS
    alu = dict(flops_per_cell_stage=flops, achieved_tflops=round(tfs, 3), peak_tflops=peak,
               frac=round(tfs / peak, 4),
               intensity_flop_per_byte=round(flops / (bytes_per_launch / cells), 2),
               ridge_flop_per_byte=round(peak * 1e3 / HBM_PEAK_GBS, 2))
    if rec is not None:
        for k in ("valu_instr_per_cell_stage", "valu_busy_frac", "wait_frac", "vgprs",
                  "scratch_bytes_per_lane"):
            if k in rec:
                alu[k] = float(rec[k])
    return roof, alu


def host_info():
    """Host CPU model and core counts (the CPU baseline's machine)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(host_cpu=model, nproc=usable, logical_cpus=os.cpu_count())


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
                       f"({dt:.1f} s wall, FP64, OpenMP over faces/cells)",
                compiler="gcc " + " ".join(O.CFLAGS), **host_info())


def cpu_single_core(case, budget_s=5.0):
    """The oracle on one host core, on a bounded sample of the same grid."""
    from oracle import oracle as O
    keep = O.num_threads()
    O.set_threads(1)
    try:
        ref = O.OracleGrid(case)
        t0 = time.perf_counter()
        ref.run(case.params, 1)
        t1 = time.perf_counter() - t0
        n = max(1, min(50, int(budget_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        ref.run(case.params, n)
        dt = time.perf_counter() - t0
    finally:
        O.set_threads(keep)
    return dict(value=round(case.ncells * n / dt, 1), unit="cell-updates/s", cores=1,
                kind="oracle", sample=f"{case.name}: {n} SSP-RK3 steps of the full grid "
                                      f"({dt:.1f} s wall, FP64, one thread)",
                compiler="gcc " + " ".join(O.CFLAGS))


# --------------------------------------------------------------------------
# batched instances and the serving trace
# --------------------------------------------------------------------------
def _drain(srv, tickets, timeout=600.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        if time.time() - t0 > timeout:
            raise RuntimeError("server did not finish in time")
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.0005)
    return out


def _plain_solve(fv, case, drop_tol, max_steps, params=None):
    """One request solved on its own: grid, upload, solve, download.  Returns
    the wall time of all of it, the wall time of the solve alone (device
    work of the steps, synchronised) and the solve's info."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = g.solve(params or case.params, drop_tol=drop_tol, max_steps=max_steps, check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.get_state()
    dt = time.perf_counter() - t0
    g.close()
    return dt, t2 - t1, info


def size_class(ncells: int) -> int:
    """floor(log2(cells)): the autotune table's size class of a grid."""
    return max(0, int(ncells).bit_length() - 1)


def tune_classes(fv, cases, cs, precisions, tune_cache):
    """Tile shapes for every (dimension, size class, precision) among the
    grids cs: the autotuner times each class once, on its first grid, and
    records the fastest shape in the table the servers and grids read.
    Returns {table key: {"rows", "ny"}} for the classes met."""
    seen = set()
    t0 = time.perf_counter()
    for c in cs:
        for pr in precisions:
            key = f"{c.ndim}d_{'fp32flux' if pr == cases.FP32_FLUX else 'fp64'}_c{size_class(c.ncells)}"
            if key in seen:
                continue
            seen.add(key)
            g = fv.Grid(c)
            g.set_state(c.state_flat())
            g.tune(cases.Params(**{**c.params.__dict__, "precision": pr}), tune_cache)
            g.close()
    with open(tune_cache) as fh:
        table = json.load(fh)
    log(f"[bench] tuned {len(seen)} size classes in {time.perf_counter() - t0:.1f} s")
    return {k: dict(rows=v["rows"], ny=v["ny"]) for k, v in sorted(table.items()) if k in seen}


def arena_for(fv, cs, slack=1.5):
    return int(sum(fv.workspace_bytes(c) for c in cs) * slack) + (64 << 20)


def bench_batched(fv, cases, tune_cache, steps=100, count=64, spl=10):
    cs = cases.batch_2d(count, seed=4, nsteps=steps)  # FP32-flux
    cells = sum(c.ncells for c in cs)
    log(f"[bench] batched {count} instances, {cells} cells, {steps} steps")
    shapes = tune_classes(fv, cases, cs, [cases.FP32_FLUX], tune_cache) if tune_cache else {}
    # plain: one instance after the other, same precision and tile shapes
    seq = seq_steps = 0.0
    for c in cs:
        dt, ds, info = _plain_solve(fv, c, 0.0, steps)
        assert info["steps"] == steps
        seq += dt
        seq_steps += ds
    srv = fv.Server(arena_bytes=arena_for(fv, cs), max_instances=count,
                    precision=cases.FP32_FLUX, steps_per_launch=spl, autotune_cache=tune_cache)
    # one untimed pass so that graphs and code objects are ready
    _drain(srv, [srv.submit(cs[0], drop_tol=0.0, max_steps=spl)])
    ts = [srv.submit(c, drop_tol=0.0, max_steps=steps) for c in cs]
    res = _drain(srv, ts)
    tm = [res[t][2]["times"] for t in ts]
    srv.close()
    assert all(res[t][0] == fv.FV_OK and res[t][2]["steps"] == steps for t in ts)
    span = max(x[2] for x in tm) - min(x[0] for x in tm)
    return dict(instances=count, cells=cells, steps=steps, precision="fp32flux",
                value=round(cells * steps / span, 1), unit="cell-updates/s",
                makespan_s=round(span, 4),
                sequential_s=round(seq, 4), sequential_value=round(cells * steps / seq, 1),
                speedup=round(seq / span, 3),
                sequential_steps_only_s=round(seq_steps, 4),
                sequential_steps_only_value=round(cells * steps / seq_steps, 1),
                speedup_vs_steps_only=round(seq_steps / span, 3),
                steps_per_launch=spl, tile_shapes=shapes,
                note="makespan: first submission to last result, uploads included; sequential_s "
                     "includes each instance's grid build, upload and download, "
                     "sequential_steps_only_s only its solve")


def _serve(fv, cases, reqs, built, arena, max_inst, spl, tune_cache, rate_scale=1.0,
           precision=None):
    srv = fv.Server(arena_bytes=arena, max_instances=max_inst,
                    precision=cases.FP64 if precision is None else precision,
                    steps_per_launch=spl, autotune_cache=tune_cache)
    _drain(srv, [srv.submit(built[0], drop_tol=0.0, max_steps=spl)])  # warm
    tickets = [None] * len(reqs)
    start = time.perf_counter()
    k = 0
    pending = set()
    done = {}
    while len(done) < len(reqs):
        now = time.perf_counter() - start
        while k < len(reqs) and reqs[k].arrival * rate_scale <= now:
            s = reqs[k].spec
            tickets[k] = srv.submit(built[k], drop_tol=s["drop_tol"], max_steps=s["max_steps"])
            pending.add(k)
            k += 1
        for q in list(pending):
            r = srv.poll(tickets[q])
            if r is not None:
                done[q] = r
                pending.discard(q)
        if now > 900:
            raise RuntimeError("serving trace did not finish")
        time.sleep(0.0002)
    tm = [done[q][2]["times"] for q in range(len(reqs))]
    srv.close()
    lat = [x[2] - x[0] for x in tm]
    span = max(x[2] for x in tm) - min(x[0] for x in tm)
    work = sum(built[q].ncells * done[q][2]["steps"] for q in range(len(reqs)))
    ok = sum(1 for q in range(len(reqs)) if done[q][0] == fv.FV_OK)
    conv = sum(1 for q in range(len(reqs)) if done[q][2]["flags"] & fv.FLAG_CONVERGED)
    capped = sum(1 for q in range(len(reqs))
                 if done[q][2]["steps"] >= reqs[q].spec["max_steps"]
                 and not done[q][2]["flags"] & fv.FLAG_CONVERGED)
    return lat, span, work, dict(ok=ok, converged=conv, capped=capped)


def _pct(xs, p):
    s = sorted(xs)
    i = min(len(s) - 1, max(0, int(math.ceil(p / 100.0 * len(s))) - 1))
    return s[i]


def bench_serving(fv, cases, tune_cache, count=256, max_steps=2000, spl=10, max_inst=32):
    """The serving trace as stated: 256 requests arriving as a Poisson stream
    at 200/s, each solved to a residual drop of 1e-8 or 2000 steps.  The
    server batches them in FP64, against plain FP64 solves one after the
    other in arrival order on the same GPU.  Supplementary: the same trace
    served in FP32-flux (whose residual stalls near the FP32 round-off of
    the fluxes, above a 1e-8 drop, so its requests mostly run to the cap),
    and the first 64 requests in FP64 at about 0.7x the measured capacity."""
    reqs = cases.serving_trace(256, seed=5, max_steps=max_steps)[:count]
    built = [cases.build_request(r, precision=cases.FP64) for r in reqs]
    arena = min(arena_for(fv, built, 1.2), 64 << 30)
    log(f"[bench] serving {count} requests, max_steps {max_steps}, arena {arena >> 20} MiB")
    shapes = tune_classes(fv, cases, built, [cases.FP64, cases.FP32_FLUX], tune_cache) \
        if tune_cache else {}
    lat, span, work, cnt = _serve(fv, cases, reqs, built, arena, max_inst, spl, tune_cache)
    log(f"[bench]   batched fp64: makespan {span:.2f} s, {cnt}")
    # plain: sequential FP64 solves in arrival order on the same GPU, with the
    # FP64 shapes of the same table
    keep = os.environ.get("FV_AUTOTUNE_CACHE")
    if tune_cache:
        os.environ["FV_AUTOTUNE_CACHE"] = tune_cache
    solve_s, steps_plain, conv_p = [], [], 0
    try:
        for q, (r, c) in enumerate(zip(reqs, built)):
            dt, _, info = _plain_solve(fv, c, r.spec["drop_tol"], r.spec["max_steps"])
            solve_s.append(dt)
            steps_plain.append(info["steps"])
            conv_p += 1 if info["flags"] & fv.FLAG_CONVERGED else 0
            if (q + 1) % 32 == 0:
                log(f"[bench]   plain: {q + 1} of {len(reqs)} solved, {sum(solve_s):.1f} s")
    finally:
        if keep is None:
            os.environ.pop("FV_AUTOTUNE_CACHE", None)
        else:
            os.environ["FV_AUTOTUNE_CACHE"] = keep
    end = 0.0
    lat_p = []
    for r, s in zip(reqs, solve_s):
        st = max(r.arrival, end)
        end = st + s
        lat_p.append(end - r.arrival)
    span_p = end - reqs[0].arrival
    work_p = sum(b.ncells * n for b, n in zip(built, steps_plain))
    log(f"[bench]   plain: makespan {span_p:.2f} s, {conv_p} converged")
    out = dict(requests=count, max_steps=max_steps, drop_tol=reqs[0].spec["drop_tol"],
               arrival_rate_per_s=200.0, completed_ok=cnt["ok"],
               converged=cnt["converged"], capped=cnt["capped"],
               batched=dict(precision="fp64", p50_s=round(_pct(lat, 50), 4),
                            p99_s=round(_pct(lat, 99), 4), makespan_s=round(span, 4),
                            value=round(work / span, 1), unit="cell-updates/s",
                            cell_steps=int(work), requests_per_s=round(count / span, 2)),
               plain=dict(precision="fp64", p50_s=round(_pct(lat_p, 50), 4),
                          p99_s=round(_pct(lat_p, 99), 4), makespan_s=round(span_p, 4),
                          value=round(work_p / span_p, 1), unit="cell-updates/s",
                          converged=conv_p, cell_steps=int(work_p),
                          requests_per_s=round(count / span_p, 2)),
               tile_shapes=shapes)
    out["throughput_ratio"] = round(out["batched"]["value"] / out["plain"]["value"], 3)
    out["request_rate_ratio"] = round(span_p / span, 3)
    # supplementary: FP32-flux batching of the same trace
    built32 = [cases.build_request(r, precision=cases.FP32_FLUX) for r in reqs]
    lat3, span3, work3, cnt3 = _serve(fv, cases, reqs, built32, arena, max_inst, spl, tune_cache,
                                      precision=cases.FP32_FLUX)
    log(f"[bench]   batched fp32-flux: makespan {span3:.2f} s, {cnt3}")
    out["batched_fp32flux"] = dict(p50_s=round(_pct(lat3, 50), 4), p99_s=round(_pct(lat3, 99), 4),
                                   makespan_s=round(span3, 4), value=round(work3 / span3, 1),
                                   cell_steps=int(work3), converged=cnt3["converged"],
                                   capped=cnt3["capped"])
    # supplementary: the first 64 requests at about 0.7x the measured capacity
    sub = min(64, count)
    cap_rate = count / span
    scale = (200.0 / (0.7 * cap_rate))
    lat2, span2, work2, cnt2 = _serve(fv, cases, reqs[:sub], built[:sub], arena, max_inst, spl,
                                      tune_cache, rate_scale=scale)
    out["low_load"] = dict(requests=sub, precision="fp64", arrival_rate_per_s=round(200.0 / scale, 2),
                           p50_s=round(_pct(lat2, 50), 4), p99_s=round(_pct(lat2, 99), 4),
                           value=round(work2 / span2, 1), converged=cnt2["converged"],
                           capped=cnt2["capped"])
    return out


# --------------------------------------------------------------------------
# rocprofv3 output -> short text summaries
# --------------------------------------------------------------------------
def _col(row, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    return None


def _counter_runs(dirs, kernel_filter):
    """{kernel: {counter: mean per dispatch, '_dur_ns', '_vgpr', ...}} over the
    counter-collection CSVs under ``dirs``."""
    per = {}
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    name = _col(row, "Kernel_Name").replace("(anonymous namespace)::", "")
                    if kernel_filter not in name:
                        continue
                    name = name.split("(")[0]
                    key = (name, d, _col(row, "Dispatch_Id"))
                    e = per.setdefault(key, {})
                    c = _col(row, "Counter_Name")
                    e[c] = e.get(c, 0.0) + float(_col(row, "Counter_Value"))
                    t0, t1 = _col(row, "Start_Timestamp"), _col(row, "End_Timestamp")
                    if t0 and t1:
                        e["_dur_ns"] = float(t1) - float(t0)
                    for k, names in (("_vgpr", ("Arch_VGPR_Count", "VGPR_Count")),
                                     ("_scratch", ("Scratch_Size",)), ("_grid", ("Grid_Size",))):
                        v = _col(row, *names)
                        if v not in (None, ""):
                            e[k] = float(v)
    agg = {}
    for (name, _, _), e in per.items():
        a = agg.setdefault(name, {"_n": {}})
        for k, v in e.items():
            a.setdefault(k, []).append(v)
    out = {}
    for name, a in agg.items():
        out[name] = {k: sum(v) / len(v) for k, v in a.items() if k != "_n"}
        out[name]["_dispatches"] = max(len(v) for k, v in a.items() if k != "_n")
    return out


def summarize(dirs, kernel_filter, out_path, command, calib=None, workload=None, precision="fp64"):
    """Kernel-trace stats (``*kernel_stats.csv``) and counter collection
    (``*counter_collection.csv``) of rocprofv3 runs as a short text file.
    ``calib`` names the runs of the same counters over a 1 GiB device copy,
    whose known traffic scales FETCH_SIZE / WRITE_SIZE (KiB) to bytes."""
    lines = ["# rocprofv3 summary", f"command: {command}", ""]
    trace_calls = trace_ns = 0.0
    for d in dirs:
        for path in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
            lines.append(f"# kernel stats ({os.path.basename(path)})")
            lines.append("| kernel | calls | total ms | avg us | min us | max us | % |")
            lines.append("|---|---|---|---|---|---|---|")
            with open(path) as fh:
                for row in csv.DictReader(fh):
                    name = _col(row, "Name").replace("(anonymous namespace)::", "").split("(")[0]
                    if kernel_filter in name:
                        trace_calls += float(_col(row, "Calls"))
                        trace_ns += float(_col(row, "TotalDurationNs"))
                    lines.append(f"| {name} | {_col(row, 'Calls')} | "
                                 f"{float(_col(row, 'TotalDurationNs'))/1e6:.3f} | "
                                 f"{float(_col(row, 'AverageNs'))/1e3:.2f} | "
                                 f"{float(_col(row, 'MinNs'))/1e3:.2f} | "
                                 f"{float(_col(row, 'MaxNs'))/1e3:.2f} | "
                                 f"{float(_col(row, 'Percentage')):.2f} |")
            lines.append("")
    cnt = _counter_runs(dirs, kernel_filter)
    if cnt:
        lines.append("# counters, mean per dispatch (FETCH_SIZE / WRITE_SIZE in KiB)")
        for name, a in sorted(cnt.items()):
            vals = ", ".join(f"{k}={v:.6g}" for k, v in sorted(a.items()) if not k.startswith("_"))
            lines.append(f"  {name}: dispatches={a['_dispatches']} dur_us={a.get('_dur_ns', 0)/1e3:.2f} "
                         f"vgpr={a.get('_vgpr')} scratch={a.get('_scratch')} grid={a.get('_grid')} {vals}")
        lines.append("")
    fetch_f = write_f = None
    if calib:
        cc = _counter_runs(calib, "copyBuffer")
        big = [a for a in cc.values() if a.get("_grid", 0) >= 65536] or list(cc.values())
        f = [a["FETCH_SIZE"] for a in big if "FETCH_SIZE" in a]
        w = [a["WRITE_SIZE"] for a in big if "WRITE_SIZE" in a]
        if f:
            fetch_f = float(1 << 30) / (max(f) * 1024.0)
        if w:
            write_f = float(1 << 30) / (max(w) * 1024.0)
        lines.append(f"# calibration: 1 GiB device copy reads FETCH_SIZE={max(f) if f else None} KiB, "
                     f"WRITE_SIZE={max(w) if w else None} KiB")
        lines.append("")
    if workload and cnt:
        from paper_2305_18057_amd import cases
        case = WORKLOADS[workload]()
        cells = case.ncells
        st = [a for n, a in cnt.items() if "stage" in n]
        def mean(k):
            v = [a[k] for a in st if k in a]
            return sum(v) / len(v) if v else None
        lines.append(f"kernel_sources_sha: "
                     f"{kernel_sources_sha(case.ndim, is_viscous(case), is_general3d(case))}")
        lines.append(f"workload: {workload}_{precision}")
        lines.append(f"cells: {cells}")
        alg = algorithmic_bytes_per_cell_step(case) * cells / 3.0
        lines.append(f"algorithmic_bytes_per_launch: {alg:.0f}")
        if trace_calls:
            # kernel execution time (first wave's start to last wave's end),
            # over every stage launch of the traced run
            lines.append(f"trace_avg_us_per_launch: {trace_ns / trace_calls / 1e3:.2f}")
        fs, ws = mean("FETCH_SIZE"), mean("WRITE_SIZE")
        if fs is not None and ws is not None and fetch_f and write_f:
            hbm = fs * 1024.0 * fetch_f + ws * 1024.0 * write_f
            lines.append(f"fetch_factor: {fetch_f:.4f}")
            lines.append(f"write_factor: {write_f:.4f}")
            lines.append(f"hbm_bytes_per_launch: {hbm:.0f}")
            lines.append(f"traffic_over_algorithmic: {hbm / alg:.3f}")
        vi = mean("SQ_INSTS_VALU")
        dur = mean("_dur_ns")
        if vi is not None:
            lines.append(f"valu_instr_per_cell_stage: {vi * 64.0 / cells:.1f}")
            if dur:
                # a wave64 VALU instruction holds its 16-lane SIMD for 4 cycles
                lines.append(f"valu_busy_frac: {vi * 4.0 / (dur * 1e-9 * 2.4e9 * 1024):.3f}")
        wa, wc = mean("SQ_WAIT_ANY"), mean("SQ_WAVE_CYCLES")
        if wa is not None and wc:
            lines.append(f"wait_frac: {wa / wc:.3f}")
        fl = mean("SQ_INSTS_VALU_FLOPS_FP64")
        if fl is not None:
            lines.append(f"fp64_flops_per_cell_stage_measured: {fl * 64.0 / cells:.1f}")
        v = mean("_vgpr")
        if v is not None:
            lines.append(f"vgprs: {v:.0f}")
        sc = mean("_scratch")
        if sc is not None:
            lines.append(f"scratch_bytes_per_lane: {sc:.0f}")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# --------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="inlet_2d", choices=sorted(WORKLOADS),
                    help="headline workload (default: the 2D inlet-like grid)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32flux"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-tune", action="store_true", help="default tile shapes, no autotuning")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the 256-request serving trace to serve (default: all)")
    ap.add_argument("--tile-cache", help="autotune table (JSON); shapes already in it are reused "
                                         "without timing (default: a fresh temporary table)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--summarize", metavar="DIRS",
                    help="comma-separated rocprofv3 CSV output folders to summarize, then exit")
    ap.add_argument("--calib", metavar="DIRS", help="with --summarize: copy-probe counter runs")
    ap.add_argument("--kernel", default="k_stage", help="kernel name filter for --summarize")
    ap.add_argument("--out", help="summary file for --summarize")
    ap.add_argument("--command", default="", help="profiling command recorded in the summary")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize.split(","), args.kernel, args.out, args.command,
                  args.calib.split(",") if args.calib else None,
                  args.workload, args.precision)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} (WORLD_SIZE={world}) is not "
              "supported: the hot path runs on a single MI355X (a large grid would shard by "
              "blocks, batches and serving by instance).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        n = 1 << 27  # 128 Mi doubles = 1 GiB
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copied 3 x {n * 8} bytes", flush=True)
        return
    from paper_2305_18057_amd import cases, fv
    fv.lib()
    tune_cache = None
    if not args.no_tune:
        tune_cache = args.tile_cache or os.path.join(tempfile.mkdtemp(prefix="fv_tune_"), "tiles.json")

    # ---- headline
    prec = cases.FP64 if args.precision == "fp64" else cases.FP32_FLUX
    case = WORKLOADS[args.workload]()
    prm = cases.Params(**{**case.params.__dict__, "precision": prec})
    log(f"[bench] headline {case.name} {args.precision} cells={case.ncells} steps={args.steps} "
        f"warmup={args.warmup}")
    g, info, wall, dev_ms, stage_ms, st = time_grid(fv, case, prm, args.steps, args.warmup, tune_cache)
    ms_per_step = dev_ms / args.steps
    value = case.ncells * args.steps / (dev_ms * 1e-3)
    roof, alu = roofline_of(case, stage_ms, args.steps, args.workload, prec == cases.FP32_FLUX)
    log(f"[bench] {value/1e9:.3f} G cell-updates/s, {ms_per_step*1e3:.1f} us/step, "
        f"stage kernel {roof['avg_launch_ms']*1e3:.1f} us -> {roof['achieved']:.0f} GB/s "
        f"({100*roof['frac']:.1f}% HBM), tile rows={st['tile_rows']} ny={st['tile_ny']}")
    g.close()
    del g
    roof["achievable_copy_gbs"] = copy_bandwidth()

    extra = {}
    props = torch.cuda.get_device_properties(0)
    extra["env"] = dict(device=torch.cuda.get_device_name(0), arch=getattr(props, "gcnArchName", ""),
                        compute_units=getattr(props, "multi_processor_count", None), hip=torch.version.hip,
                        torch=torch.__version__)
    rep = repeat_timing(fv, case, prm, args.steps, 5, tune_cache)
    extra["repeats"] = rep
    log(f"[bench] median of {rep['reps']} runs from the restored initial state: "
        f"{rep['median_ms_per_step']*1e3:.1f} us/step")
    if not args.no_extra:
        others = [("inlet_2d", cases.inlet_2d, cases.FP64, args.steps),
                  ("inlet_2d", cases.inlet_2d, cases.FP32_FLUX, args.steps),
                  ("blobs_3d", cases.blobs_3d, cases.FP64, 50),
                  ("blobs_3d", cases.blobs_3d, cases.FP32_FLUX, 50),
                  ("inlet_2d_ns", cases.inlet_2d_ns, cases.FP64, args.steps),
                  ("inlet_2d_ns", cases.inlet_2d_ns, cases.FP32_FLUX, args.steps),
                  ("curv3d_mms", WORKLOADS["curv3d_mms"], cases.FP64, 20),
                  ("curv3d_mms", WORKLOADS["curv3d_mms"], cases.FP32_FLUX, 20)]
        for wl, mk, pr, steps in others:
            name = f"{wl}_{'fp64' if pr == cases.FP64 else 'fp32flux'}"
            if wl == args.workload and pr == prec:
                continue
            c = mk()
            p = cases.Params(**{**c.params.__dict__, "precision": pr})
            log(f"[bench] extra {name} cells={c.ncells} steps={steps}")
            gx, ix, wx, dx, sx, stx = time_grid(fv, c, p, steps, 5, tune_cache)
            rx, ax = roofline_of(c, sx, steps, wl, pr == cases.FP32_FLUX)
            extra[name] = dict(value=round(c.ncells * steps / (dx * 1e-3), 1),
                               ms_per_step=round(dx / steps, 5), roofline=rx, alu=ax,
                               tile=dict(rows=stx["tile_rows"], ny=stx["tile_ny"],
                                         tiles=stx["tiles"], blocks=stx["launch_blocks"]))
            log(f"[bench]   {extra[name]['value']/1e9:.3f} G cell-updates/s, "
                f"{rx['achieved']:.0f} GB/s ({100*rx['frac']:.1f}% HBM), "
                f"rows={stx['tile_rows']} ny={stx['tile_ny']}")
            gx.close()
            del gx
        extra["rk_schemes"] = bench_rk_schemes(fv, cases, tune_cache, args.steps)
        extra["hetero"] = bench_hetero(fv, cases, tune_cache)
        extra["hetero_ns"] = bench_hetero(fv, cases, tune_cache, viscous=True)
        tc = tune_cache or os.path.join(tempfile.mkdtemp(prefix="fv_tune_"), "tiles.json")
        extra["batched_64"] = bench_batched(fv, cases, None if args.no_tune else tc)
        b = extra["batched_64"]
        log(f"[bench]   batched {b['value']/1e9:.3f} G cell-updates/s vs sequential "
            f"{b['sequential_value']/1e9:.3f} G ({b['speedup']}x)")
        extra["serving"] = bench_serving(fv, cases, None if args.no_tune else tc,
                                         count=args.serving_requests)
        s = extra["serving"]
        log(f"[bench]   serving p50 {s['batched']['p50_s']} s p99 {s['batched']['p99_s']} s, "
            f"{s['batched']['value']/1e9:.3f} G/s vs plain p50 {s['plain']['p50_s']} s "
            f"p99 {s['plain']['p99_s']} s {s['plain']['value']/1e9:.3f} G/s; "
            f"{s['converged']} converged, {s['capped']} at the step cap")

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU reference on a bounded sample")
        cpu = cpu_baseline(case)
        log(f"[bench] cpu {cpu['value']/1e6:.2f} M cell-updates/s on {cpu['cores']} threads")
        extra["cpu_single_core"] = cpu_single_core(case)
        log(f"[bench] cpu one core {extra['cpu_single_core']['value']/1e6:.2f} M cell-updates/s")

    if args.workload == "inlet_2d_ns":
        desc = ("inlet_2d_ns: 2D Navier-Stokes, 4 blocks x 512x256 cells on the sheared wavy "
                "inlet-like curvilinear mesh, Mach 4 inflow (p=12270 Pa, T=217 K), no-slip walls, "
                "extrapolation outflow, mu=1.5e-2 Pa s, Pr=0.72, MUSCL-minmod + Roe + viscous flux, "
                "SSP-RK3, CFL 0.5")
    elif args.workload == "curv3d_mms":
        desc = ("curv3d_mms: 3D Euler with a manufactured solution's source, 192^3 cells in two "
                "linked blocks of a smoothly deformed periodic box (curvilinear hexahedra), "
                "MUSCL-minmod + Roe - |Omega| S_h, SSP-RK3, CFL 0.5")
    elif args.workload == "inlet_2d":
        desc = ("inlet_2d: 2D Euler, 4 blocks x 512x256 cells on the sheared wavy inlet-like "
                "curvilinear mesh, Mach 4 inflow (p=12270 Pa, T=217 K), slip walls, extrapolation "
                "outflow, MUSCL-minmod + Roe, SSP-RK3, CFL 0.5")
    else:
        desc = ("blobs_3d: 3D Euler, one uniform 256^3 block, Mach 2 free stream with 16 seeded "
                "Gaussian density blobs, supersonic inflow / extrapolation outflow, periodic "
                "transverse faces, MUSCL-minmod + Roe, SSP-RK3, CFL 0.5")
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
        "dtype": "f64" if prec == cases.FP64 else "f32-flux/f64-state",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "cells": case.ncells,
            "precision": args.precision,
            "tile_rows": st["tile_rows"],
            "tile_ny": st["tile_ny"],
            "tiles": st["tiles"],
            "launch_blocks": st["launch_blocks"],
            "autotuned": tune_cache is not None,
        },
        "cell_stage_updates_per_s": round(3 * value, 1),
        "ssspnt": round(1e-6 * case.ncells * 3 * args.steps / (dev_ms * 1e-3), 2),
        "roofline": roof,
        # the 256^3 grid's stage kernel: its 2.1 GB working set does not fit the
        # 256 MB last-level cache, so this is the DRAM-backed HBM figure
        "roofline_blobs_3d": (dict(extra["blobs_3d_fp64"]["roofline"], workload="blobs_3d_fp64")
                              if "blobs_3d_fp64" in extra else None),
        "alu": alu,
        "cpu_baseline": cpu,
        "extra": extra,
        "wall_s_timed": round(wall, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
