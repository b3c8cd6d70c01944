"""Throughput of the MI355X Oregonator stepper.

Default workload (the scale case): a 16384x16384 FP32 grid with phi ~ U[0.04,
0.08) i.i.d. per cell, u = v = 0 with 64 r=5 stimulus disks at t=0, and 2,000
forward-Euler steps of Eq. (1) with T steps per launch.  One benchmark step =
one whole run of the workload.  Inputs are resident in HBM before the timed
region; the state is reset on the device at the start of every run.

Prints one JSON line: GCell-updates/s (whole job), the roofline of the
dominant kernel (its average launch measured with HIP events on the stream it
runs on), the one-step kernel's HBM rate beside a plain copy kernel and the
runtime's device-to-device copy, and the FP64 CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1]
    python bench.py --workload circuit     # 4096^2 circuit map, 10,000 steps
    python bench.py --workload batch       # 512-grid sweep, 5,000 steps
    python bench.py --workload surrogate   # learned coarse stepper on 2048^2
    python bench.py --workload variants    # 16384^2: every launch shape, FP32 and FP64
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GCell-updates/s (FP32 Oregonator) + %HBM peak; surrogate speedup at <=1-cell error"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_ALU_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz, unpacked
FLOP_PER_UPDATE = 21            # canonical per-cell expression, divide counted once
BYTES_PER_CELL_LAUNCH = 20      # read u, v, phi (12 B) + write u', v' (8 B), FP32


def load_traffic(key: str):
    """Per-launch HBM bytes from rocprofv3 counters, if they were taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(key)
    from paper_1901_06535_amd.profile_kernels import source_hash
    if not ent or ent.get("source_hash") != source_hash():
        return None
    return ent


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, target_s: float = 24.0, runs: int = 3):
    """The FP64 oracle on the same workload, all host cores: `runs` timed
    samples of the same number of steps from the workload's start (stimuli
    at step 0 applied), about target_s seconds in all; the median rate."""
    import oracle
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params)
    run.stimulate([(s.cx, s.cy, s.r) for s in wl.stimuli if s.step == 0])
    t0 = time.perf_counter()
    run.advance(1)
    probe = time.perf_counter() - t0
    n = max(1, int(target_s / runs / max(probe, 1e-6)))
    rates = []
    for _ in range(runs):
        t0 = time.perf_counter()
        run.advance(n)
        rates.append(wl.nx * wl.ny * n / (time.perf_counter() - t0) / 1e9)
    del run
    return {"value": round(statistics.median(rates), 4), "unit": "GCell-updates/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": "FP64 oracle (C, OpenMP over rows) on the same %dx%d workload: median of "
                      "%d runs of %d steps each from its start (%s)"
                      % (wl.nx, wl.ny, runs, n, ", ".join("%.3f" % r for r in rates)),
            "cpu": cpu_model(), "nproc": os.cpu_count()}


def _hip_memcpy_d2d():
    """hipMemcpyAsync of the HIP runtime (device to device), for the
    bandwidth ceiling next to the library's own copy kernel."""
    lib = ctypes.CDLL("libamdhip64.so")
    fn = lib.hipMemcpyAsync
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                   ctypes.c_void_p]
    return fn


def copy_ceilings(stream, nbytes: int = 2 << 30, reps: int = 10):
    """Read+write GB/s of the library's copy kernel and of hipMemcpyAsync
    (device to device) on `nbytes` buffers, HIP events on `stream`."""
    import torch
    from paper_1901_06535_amd import rdc
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    memcpy = _hip_memcpy_d2d()
    out = {}
    for name in ("copy_kernel", "hipMemcpyAsync_d2d"):
        def go():
            if name == "copy_kernel":
                rdc.rdc_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
            else:
                rc = memcpy(dst.data_ptr(), src.data_ptr(), nbytes, 3, stream.cuda_stream)
                if rc != 0:
                    raise RuntimeError("hipMemcpyAsync failed: %d" % rc)
        go()
        e0, e1 = _events()
        e0.record(stream)
        for _ in range(reps):
            go()
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / reps
        out[name + "_GBs"] = round(2 * nbytes / t / 1e9, 1)
    del src, dst
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--T", type=int, default=0, help="steps per launch (0 = autotune)")
    ap.add_argument("--rows", type=int, default=0, help="tile rows (0 = autotune)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-per-grid", action="store_true",
                    help="batch workloads: skip the per-grid-context baseline")
    ap.add_argument("--workload", default="uniform",
                    choices=("uniform", "circuit", "batch", "batch_small", "surrogate", "variants"),
                    help="uniform: 16384^2, phi ~ U[0.04, 0.08), 64 disks, 2,000 steps "
                         "(default); circuit: 4096^2 circuit map, 256 disks, 10,000 steps; "
                         "batch: 512-grid sweep, 5,000 steps, batched vs per-grid; surrogate: "
                         "learned coarse stepper trained on 512^2 patches, run on a 2048^2 "
                         "circuit for 50,000 steps against the plain stepper; variants: every "
                         "launch shape on the 16384^2 grid, FP32 and FP64")
    ap.add_argument("--train-pairs", type=int, default=20000,
                    help="surrogate: (t, t+50) training pairs of 512^2 patches")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py measures one GPU: the library has no multi-GPU path "
                 "(--gpus %d requested)" % args.gpus)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "batch_small":
        return bench_batch(args, small=True)
    if args.workload == "variants":
        return bench_variants(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    return bench_plain(args)


def bench_plain(args):
    """The plain stepper on one grid: the uniform 16384^2 workload (default)
    or the 4096^2 circuit workload."""
    import torch
    from paper_1901_06535_amd import inputs, rdc

    if not os.path.exists(rdc.LIB_PATH):
        from paper_1901_06535_amd import build
        build.build()
    if args.workload == "circuit":
        wl = inputs.circuit(n=4096, seed=1002, steps=10000, ndisks=256)
        label = "circuit_%dx%d_%dsteps" % (wl.nx, wl.ny, wl.steps)
    else:
        wl = inputs.uniform_random_phi(n=16384, seed=1003, steps=2000, ndisks=64)
        label = "uniform_phi_%dx%d_%dsteps" % (wl.nx, wl.ny, wl.steps)
    sim = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
    sim.set_phi(wl.phi)
    dev = torch.device("cuda")
    u0 = torch.zeros((wl.ny, wl.nx), dtype=torch.float32, device=dev)
    v0 = torch.zeros_like(u0)
    stream = sim.stream

    def reset():
        sim.write(u0, v0)

    def one_run():
        reset()
        start = sim.step_index
        sched = [(s.step + start, s.cx, s.cy, s.r) for s in wl.stimuli]
        sim.run_schedule(sched, start + wl.steps)

    def time_steps(T, rows, n):
        sim.set_block(T)
        if rows:
            sim.set_tile_rows(rows)
        reset()
        sim.step(2 * T)
        e0, e1 = _events()
        e0.record(stream)
        sim.step(n)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1e3

    if args.T and args.rows:
        T, rows = args.T, args.rows
        tune = {}
    else:
        rec = sim.autotune(Ts=(args.T,) if args.T else (6, 7, 8, 9, 10, 11, 12),
                           rows=(args.rows,) if args.rows else (48, 56, 64, 80,
                                                                rdc.RDC_TILE_STREAM),
                           launches=24 if wl.nx > 8192 else 48, use_cache=False)
        T, rows, tune = rec["T"], rec["rows"], rec["table"]
    sim.set_block(T)
    sim.set_tile_rows(rows)

    for _ in range(args.warmup):
        one_run()
    torch.cuda.synchronize()
    e0, e1 = _events()
    marks = [_events()[0] for _ in range(args.steps + 1)]   # per-run boundaries
    t_wall = time.perf_counter()
    e0.record(stream)
    marks[0].record(stream)
    for k in range(args.steps):
        one_run()
        marks[k + 1].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    run_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps))
    t = e0.elapsed_time(e1) / 1e3
    cells = wl.nx * wl.ny
    updates = cells * wl.steps * args.steps
    value = updates / t / 1e9

    # -- dominant kernel: average launch of the T-step kernel, HIP events on its stream
    nlaunch = 40 if cells > (1 << 26) else 200
    t_k = time_steps(T, rows, T * nlaunch) / nlaunch
    flops = FLOP_PER_UPDATE * cells * T
    achieved_tf = flops / t_k / 1e12
    achieved_bw = BYTES_PER_CELL_LAUNCH * cells / t_k / 1e9
    from paper_1901_06535_amd.profile_kernels import traffic_key
    kname = ("k_stream<T=%d>" % T) if rows == rdc.RDC_TILE_STREAM else (
        "k_stepT<T=%d,rows=%d>" % (T, rows))
    traf = load_traffic(traffic_key(kname, wl.nx))
    alu = {"bound": "alu", "achieved": round(achieved_tf, 2), "peak": FP32_ALU_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(achieved_tf / FP32_ALU_PEAK_TFLOPS, 4),
           "traffic": traf["bytes_per_launch"] if traf else None}
    hbm_eff = {"bound": "hbm", "achieved": round(achieved_bw, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(achieved_bw / HBM_PEAK_GBS, 4),
               "traffic": traf["bytes_per_launch"] if traf else None}
    # The binding roof is the one whose attainable rate is lower, i.e. the
    # one the kernel reaches the larger fraction of.
    roof = alu if alu["frac"] >= hbm_eff["frac"] else hbm_eff
    other = hbm_eff if roof is alu else alu

    # -- the one-step kernel (20 B per cell-update) against the copy ceilings
    n1 = 20 if cells > (1 << 26) else 200
    t1 = time_steps(1, 0, n1) / n1
    one_step = {"kernel": "k_step1<float>", "launch_ms": round(1e3 * t1, 4),
                "achieved_GBs": round(BYTES_PER_CELL_LAUNCH * cells / t1 / 1e9, 1),
                "gcells": round(cells / t1 / 1e9, 1)}
    one_step["frac_of_peak"] = round(one_step["achieved_GBs"] / HBM_PEAK_GBS, 4)
    one_step.update(copy_ceilings(stream))

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GCell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": label, "grid": [wl.nx, wl.ny], "steps_per_run": wl.steps,
                   "stimuli": len(wl.stimuli), "steps_per_launch": T, "tile_rows": rows,
                   "parallelism": "single GPU"},
        "roofline": dict(roof, kernel=kname,
                         launch_ms=round(1e3 * t_k, 4),
                         traffic_GBs=round(traf["bytes_per_launch"] / t_k / 1e9, 1) if traf else None,
                         algorithmic="%d FLOP/update x %d updates; %d B/cell x %d cells"
                                     % (FLOP_PER_UPDATE, cells * T, BYTES_PER_CELL_LAUNCH, cells)),
        "roofline_other": other,
        "one_step_kernel": one_step,
        "tuning_us_per_step": tune,
        "run_ms": {"median": round(run_ms[len(run_ms) // 2], 3), "min": round(run_ms[0], 3),
                   "max": round(run_ms[-1], 3),
                   "median_value": round(cells * wl.steps / (run_ms[len(run_ms) // 2] / 1e3) / 1e9,
                                         2)},
        "wall_s": round(wall, 3),
    }
    sim.close()
    del u0, v0
    torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_batch(args, small=False):
    """512 independent grids (sides log-uniform in [64, 1024], own eps and
    phi_excitable, channel lattices, 1-4 disks at t=0), 5,000 steps: one
    batched launch per T steps for the tiled grids and one whole-grid launch
    for the small ones, replayed from a HIP graph; against the same batch
    with every grid tiled, and against stepping each grid through its own
    single-grid context.  With `small`, 1,024 grids with sides in [64, 128]
    (every one on the whole-grid path)."""
    import torch
    from paper_1901_06535_amd import inputs, rdc

    if not os.path.exists(rdc.LIB_PATH):
        from paper_1901_06535_amd import build
        build.build()
    if small:
        sims, steps = inputs.batch_sweep(count=1024, seed=1006, smin=64, smax=128)
    else:
        sims, steps = inputs.batch_sweep(count=512, seed=1004)
    cells = sum(s.nx * s.ny for s in sims)
    b = rdc.BatchSim([(s.nx, s.ny, s.params) for s in sims])
    for i, s in enumerate(sims):
        b.set_phi(i, s.phi)
    disks = [(i, d.cx, d.cy, d.r) for i, s in enumerate(sims) for d in s.stimuli]
    stream = b.stream.cuda_stream
    zeros = torch.zeros(b.pool_elems, dtype=torch.float32, device="cuda")
    nbytes = 4 * b.pool_elems

    def reset():
        # u, v := 0 in every grid with the library's copy kernel, then the disks
        for plane in (b.planes[0], b.planes[2]):
            rdc.rdc_copy(plane.data_ptr(), zeros.data_ptr(), nbytes, stream)
        b.stimulate(disks)

    # autotune the tiled grids' launch shape on the sweep's shapes (nothing
    # to tune when every grid is on the whole-grid path)
    if b.resident_count() < len(sims):
        rec = b.autotune(launches=24, use_cache=False)
        T, rows, tune = rec["T"], rec["rows"], rec["table"]
    else:
        T, rows, tune = 8, 56, None
        b.set_block(T, rows)
    g = b.capture(steps)
    for _ in range(args.warmup):
        reset()
        g.launch()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(b.stream)
    for _ in range(args.steps):
        reset()
        g.launch()
    e1.record(b.stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    value = cells * steps * args.steps / t / 1e9
    resident = b.resident_count()
    diverged = []
    for i in range(len(sims)):
        try:
            b.read(i)
        except rdc.RdcError as e:
            if e.status != rdc.RDC_E_NONFINITE:
                raise
            diverged.append(i)
    bu, bv = (t.clone() for t in b.current())       # the batch's final states (pooled)
    g.close()
    # the same batch with every grid tiled (one run, after a warm-up run), at
    # its own best launch shape
    b.set_resident(0)
    if tune is None:
        b.autotune(launches=24, use_cache=False)
    g = b.capture(steps)
    reset()
    g.launch()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(b.stream)
    reset()
    g.launch()
    e1.record(b.stream)
    torch.cuda.synchronize()
    t_tiled = e0.elapsed_time(e1) / 1e3
    tu, tv = b.current()

    def grid(plane, i):
        nx, ny, pitch, off = b.shapes[i]
        return plane[off:off + ny * pitch].view(ny, pitch)[:, :nx]
    tiled_same = all(torch.equal(grid(tu, i), grid(bu, i)) and torch.equal(grid(tv, i), grid(bv, i))
                     for i in range(len(sims)) if i not in diverged)
    g.close()
    b.close()
    del zeros

    # per-grid baseline: each grid through its own context, same T and tile
    # rows; contexts, phi and disks are set up before the timed region
    ctxs = []
    for s in ([] if args.no_per_grid else sims):
        sim = rdc.Sim(s.nx, s.ny, s.params, "fp32")
        sim.set_phi(s.phi)
        sim.set_block(T)
        sim.set_tile_rows(rows)
        sim.stimulate([(d.cx, d.cy, d.r) for d in s.stimuli])
        ctxs.append(sim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = _events()
    e0.record()
    for sim in ctxs:
        sim.step(steps)
    e1.record()
    torch.cuda.synchronize()
    t_single = e0.elapsed_time(e1) / 1e3 if ctxs else float("nan")
    wall_single = time.perf_counter() - t0
    # every finite grid must end bit-identical to the same grid stepped alone
    same = 0
    for i, (sim, (nx, ny, pitch, off)) in enumerate(zip(ctxs, b.shapes)):
        if i in diverged:
            continue
        su, sv = sim.current()
        gu = bu[off:off + ny * pitch].view(ny, pitch)[:, :nx]
        gv = bv[off:off + ny * pitch].view(ny, pitch)[:, :nx]
        same += int(torch.equal(su, gu) and torch.equal(sv, gv))
    for sim in ctxs:
        sim.close()
    single = cells * steps / t_single / 1e9
    per_grid = None if not ctxs else {
        "value": round(single, 2), "unit": "GCell-updates/s", "seconds": round(t_single, 3),
        "wall_s": round(wall_single, 3), "speedup": round(value / single, 2),
        "finite_grids_bitwise_equal": "%d/%d" % (same, len(sims) - len(diverged))}
    ach = 21.0 * cells * steps * args.steps / t / 1e12
    if resident == len(sims):
        # one whole-grid launch per run: ALU-bound (no HBM traffic between steps)
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": 78.6, "unit": "TFLOP/s",
                "frac": round(ach / 78.6, 4), "traffic": None, "kernel": "k_batch_resident",
                "launch_ms": round(1e3 * t / args.steps, 3),
                "algorithmic": "21 FLOP/update x %d cells x %d steps per launch" % (cells, steps)}
    else:
        # the whole graph replay (batched T-step launches, the small grids'
        # whole-grid launch beside them): the run's FLOP rate
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": 78.6, "unit": "TFLOP/s",
                "frac": round(ach / 78.6, 4), "traffic": None,
                "kernel": "whole run (%s, k_batch_resident)"
                          % ("k_batch_stream<T=%d>" % T if rows == 1 else
                             "k_batch_stepT<T=%d,rows=%d>" % (T, rows)),
                "run_ms": round(1e3 * t / args.steps, 3),
                "algorithmic": "21 FLOP/update x %d cells x %d steps per run" % (cells, steps)}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GCell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_sweep_%s%d_grids_%dsteps"
                               % ("small_" if small else "", len(sims), steps),
                   "grids": len(sims), "cells": cells, "steps_per_run": steps,
                   "steps_per_launch": T, "tile_rows": rows, "graph": True,
                   "whole_grid_lds_grids": resident, "parallelism": "single GPU"},
        "all_tiled": {"value": round(cells * steps / t_tiled / 1e9, 2), "seconds": round(t_tiled, 4),
                      "finite_grids_bitwise_equal": tiled_same},
        "roofline": roof,
        "per_grid_baseline": per_grid,
        "diverged_grids": len(diverged),
        "diverged_eps_max": round(max(sims[i].params["eps"] for i in diverged), 5) if diverged else None,
        "tuning_us_per_step": tune,
    }
    print(json.dumps(out), flush=True)


def bench_variants(args):
    """16384^2, phi ~ U[0.04, 0.08), 64 disks, 2,000 steps: every launch
    shape of the FP32 kernels, and the FP64 kernels on the same inputs."""
    import torch
    from paper_1901_06535_amd import inputs, rdc

    if not os.path.exists(rdc.LIB_PATH):
        from paper_1901_06535_amd import build
        build.build()
    wl = inputs.uniform_random_phi(n=16384, seed=1003, steps=2000)
    sim = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
    sim.set_phi(wl.phi)
    zeros = torch.zeros((wl.ny, wl.nx), dtype=torch.float32, device="cuda")
    disks = [(s.cx, s.cy, s.r) for s in wl.stimuli]
    res = {}
    for T, rows in ((1, 0), (8, 48), (8, 56), (8, 64), (10, 64), (11, 64), (12, 56), (12, 64),
                    (8, rdc.RDC_TILE_STREAM), (10, rdc.RDC_TILE_STREAM),
                    (11, rdc.RDC_TILE_STREAM), (12, rdc.RDC_TILE_STREAM)):
        sim.set_block(T)
        if rows:
            sim.set_tile_rows(rows)
        sim.write(zeros, zeros)
        sim.stimulate(disks)
        sim.step(8)
        e0, e1 = _events()
        e0.record(sim.stream)
        sim.step(wl.steps)
        e1.record(sim.stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        res["T%d_r%d" % (T, rows)] = wl.nx * wl.ny * wl.steps / t / 1e9
    sim.close()
    # The FP64 variants on the same inputs: one step per launch (40 B per
    # cell-update, HBM-bound), T steps per launch on 128-column tiles, and
    # the FP64 row pipelines (rows 1).
    s64 = rdc.Sim(wl.nx, wl.ny, wl.params, "fp64")
    s64.set_phi(wl.phi)
    z64 = torch.zeros((wl.ny, wl.nx), dtype=torch.float64, device="cuda")
    n64 = 480
    res64 = {}
    for T, rows in ((1, 0), (4, 56), (6, 56), (8, 48), (8, 56), (8, 64),
                    (6, rdc.RDC_TILE_STREAM), (8, rdc.RDC_TILE_STREAM)):
        s64.set_block(T)
        s64.set_tile_rows(rows)
        s64.write(z64, z64)
        s64.stimulate(disks)
        s64.step(8)
        e0, e1 = _events()
        e0.record(s64.stream)
        s64.step(n64)
        e1.record(s64.stream)
        e1.synchronize()
        res64["T%d_r%d" % (T, rows)] = wl.nx * wl.ny * n64 / (e0.elapsed_time(e1) / 1e3) / 1e9
    s64.close()
    fp64 = res64["T1_r0"]
    best64 = max(res64, key=res64.get)
    best = max(res, key=res.get)
    t1 = res["T1_r0"]
    out = {
        "metric": METRIC, "value": round(res[best], 2), "unit": "GCell-updates/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uniform_phi_16384x16384_2000steps_variants", "best": best},
        "per_variant_gcells": {k: round(v, 1) for k, v in res.items()},
        "one_step_kernel_hbm": {"achieved_GBs": round(t1 * BYTES_PER_CELL_LAUNCH, 1),
                                "peak_GBs": HBM_PEAK_GBS,
                                "frac": round(t1 * BYTES_PER_CELL_LAUNCH / HBM_PEAK_GBS, 4)},
        "fp64_one_step_kernel": {"gcells": round(fp64, 1), "achieved_GBs": round(fp64 * 40, 1),
                                 "frac": round(fp64 * 40 / HBM_PEAK_GBS, 4), "steps": n64},
        "fp64_per_variant_gcells": {k: round(v, 1) for k, v in res64.items()},
        "fp64_best": best64,
    }
    print(json.dumps(out), flush=True)


MFMA_BF16_PEAK_TFLOPS = 2500.0    # MI355X dense bf16


def bench_surrogate(args):
    """Learned coarse stepper (K = 50 steps per network step): trained on the
    GPU on (t, t+50) pairs of 512^2 patches that the plain stepper generates
    from random circuits (batch 4, Adam, half the iterations on the network's
    own one-step predictions as inputs), then run on a 2048^2 circuit for
    50,000 steps with a plain-stepper check every 10 network steps and
    fallback when the front error exceeds one cell.  Reports its throughput
    and speedup against the plain stepper (at its autotuned launch shape) on
    the same grid and schedule twice: with every network step checked (the
    run then continues from the plain result of every window, and its front
    stays within one cell of the plain trajectory: the headline value), and
    with every tenth step checked, at the front error a lock-step plain run
    measures; and the roofline of the heaviest convolution."""
    import torch
    from paper_1901_06535_amd import inputs, rdc, surrogate as sg

    if not os.path.exists(rdc.LIB_PATH):
        from paper_1901_06535_amd import build
        build.build()
    K, batch, patch, pushforward = 50, 4, 512, 0.5
    iters = max(1, args.train_pairs // batch)
    net = sg.UNet(seed=0)
    tr = sg.Trainer(net, n=patch, batch=batch, K=K, seed=100, pushforward=pushforward)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        losses.append(tr.step(1e-3 * (0.1 ** (it / iters))))
        if (it + 1) % 500 == 0:
            print("# train iter %d/%d loss %.3g (%.1f s)" % (it + 1, iters,
                  float(np.mean(losses[-500:])), time.perf_counter() - t0), file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    tr.close()
    # held-out pairs: network vs persistence
    ev = sg.Trainer(net, n=patch, batch=batch, K=K, seed=900000)
    l_net = l_per = 0.0
    for _ in range(8):
        u, v, phi, ut, vt = ev.pair()
        sg.prep(net, ev.ws, u, v, phi, ev.pitch, ev.plane)
        sg.forward(net, ev.ws)
        l_net += sg.loss_and_grad(net, ev.ws, u, v, ut, vt, ev.pitch, ev.plane)
        ev.ws.a["head"].zero_()
        l_per += sg.loss_and_grad(net, ev.ws, u, v, ut, vt, ev.pitch, ev.plane)
    ev.close()

    wl = inputs.circuit(n=2048, seed=1005, steps=50000, ndisks=64, tile=256, disk_order="time")
    zeros = torch.zeros((wl.ny, wl.nx), dtype=torch.float32, device="cuda")
    # plain stepper on the same schedule
    sim = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
    sim.set_phi(wl.phi)
    plain_shape = sim.autotune()          # the plain stepper at its best launch shape

    def plain_run():
        sim.write(zeros, zeros)
        start = sim.step_index
        sim.run_schedule([(s.step + start, s.cx, s.cy, s.r) for s in wl.stimuli],
                         start + wl.steps)
    plain_run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_run()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_u = sim.current()[0].clone()

    def coarse_run(track, check_every=10):
        cs = sg.CoarseStepper(net, wl.nx, wl.ny, wl.params, wl.phi, K=K, check_every=check_every,
                              track=track)
        cs.write(zeros, zeros)
        torch.cuda.synchronize()
        t = time.perf_counter()
        cs.advance_to(wl.steps, wl.stimuli)
        torch.cuda.synchronize()
        return cs, time.perf_counter() - t
    cs, _ = coarse_run(False)          # warm-up
    cs.close()
    cs, t_coarse = coarse_run(False)
    stats = dict(cs.stats)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    rdc.nn("front_check", cs.current()[0].data_ptr(), sim.current()[0].data_ptr(), cs.pitch,
           wl.nx, wl.ny, 0.5, cnt.data_ptr(), cs.net.stream.cuda_stream)
    final_off = int(cnt.item())
    # heaviest convolution: events around each launch of a few forwards (the
    # inference form the coarse stepper runs), and around each whole forward
    evs, whole = {}, []
    cu, cv = cs.sim.current()
    uo, vo = torch.empty_like(cu), torch.empty_like(cv)
    for _ in range(5):
        w0, w1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0.record(net.stream)
        sg.forward_planes(net, cs.ws, cu.data_ptr(), cv.data_ptr(), cs.sim.planes[4].data_ptr(),
                          cs.pitch, cs.plane, events=evs,
                          predict=(uo.data_ptr(), vo.data_ptr(), wl.params))
        w1.record(net.stream)
        whole.append((w0, w1))
    torch.cuda.synchronize()
    whole_ms = float(np.mean([a.elapsed_time(b) for a, b in whole[1:]]))
    per = {n: float(np.mean([a.elapsed_time(b) for a, b in evs[n][1:]])) / 1e3 for n in evs}
    heavy = max(per, key=per.get)
    fl = sg.conv_flops(heavy, cs.ws)
    fwd_s = sum(per.values())
    cs.close()
    cs_tr, _ = coarse_run(True)
    tracked = dict(cs_tr.stats)
    cs_tr.close()
    # Every network step checked: the run continues from the plain result of
    # every window, so its front error against the plain trajectory is the
    # one setting that keeps it within one cell throughout (tracked below).
    cs1, t_coarse1 = coarse_run(False, check_every=1)
    stats1 = dict(cs1.stats)
    cs1.close()
    cs1_tr, _ = coarse_run(True, check_every=1)
    tracked1 = dict(cs1_tr.stats)
    cs1_tr.close()
    sim.close()
    cells = wl.nx * wl.ny
    value = cells * wl.steps / t_coarse1 / 1e9
    achieved = fl / per[heavy] / 1e12
    nbytes = sg.conv_bytes(heavy, cs.ws)
    achieved_bw = nbytes / per[heavy] / 1e9
    # The heaviest layer against both roofs; a 32-output-channel layer moves
    # ~200 FLOP per byte, below the bf16 ridge (2500 / 8 = 312), so its own
    # roof is HBM.  The bound reported is the roof it comes closest to.
    px_heavy = cs.ws._hw(heavy)[0] * cs.ws._hw(heavy)[1] * cs.ws.N
    mfma = {"bound": "mfma", "achieved": round(achieved, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4),
            "traffic": None}
    hbm = {"bound": "hbm", "achieved": round(achieved_bw, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved_bw / HBM_PEAK_GBS, 4), "traffic": None}
    roof, other = (hbm, mfma) if hbm["frac"] >= mfma["frac"] else (mfma, hbm)
    roof = dict(roof, kernel="k_conv3x3 (%s)" % heavy, launch_ms=round(1e3 * per[heavy], 4),
                algorithmic="%d FLOP and %d B per launch (2 x 9 x cin x cout FLOP and the "
                            "input read + output written once per pixel, %d pixels)"
                            % (fl, nbytes, px_heavy))
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GCell-updates/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * t_coarse1, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 network (fp32 accumulate) + f32 plain checks", "data": "synthetic",
        "config": {"workload": "surrogate_circuit_2048x2048_50000steps", "K": K,
                   "check_every": 10, "train_pairs": iters * batch, "train_patch": patch,
                   "stimuli": len(wl.stimuli), "last_stimulus_step": max(s.step for s in wl.stimuli),
                   "parallelism": "single GPU"},
        # value / ms_per_step: the setting whose front stays within one cell
        # of the plain trajectory (every network step checked)
        "speedup_vs_plain_at_le_1_cell": round(t_plain / t_coarse1, 4),
        "at_le_1_cell": {"check_every": 1, "seconds": round(t_coarse1, 4), "coarse_stats": stats1,
                         "tracked_windows": tracked1["tracked_windows"],
                         "windows_more_than_1_cell_off": tracked1["windows_off"],
                         "max_cells_more_than_1_cell_off": tracked1["max_cells_off"]},
        "at_measured_error": {"check_every": 10, "seconds": round(t_coarse, 4),
                              "speedup_vs_plain": round(t_plain / t_coarse, 4),
                              "coarse_stats": stats,
                              "tracked_windows": tracked["tracked_windows"],
                              "windows_more_than_1_cell_off": tracked["windows_off"],
                              "max_cells_more_than_1_cell_off": tracked["max_cells_off"],
                              "final_cells_more_than_1_cell_off": final_off},
        "plain": {"seconds": round(t_plain, 4), "value": round(cells * wl.steps / t_plain / 1e9, 2),
                  "unit": "GCell-updates/s", "steps_per_launch": plain_shape["T"],
                  "tile_rows": plain_shape["rows"]},
        "training": {"seconds": round(t_train, 2), "iters": iters, "batch": batch,
                     "pushforward": pushforward,
                     "pairs_per_s": round(iters * batch / t_train, 1),
                     "loss_first_100": float(np.mean(losses[:100])),
                     "loss_last_100": float(np.nanmean(losses[-100:])),
                     "dropped_batches_nonfinite_plain": tr.dropped_batches,
                     "skipped_iters_nonfinite_loss": tr.skipped_iters,
                     "held_out_loss_net": l_net / 8, "held_out_loss_persistence": l_per / 8},
        "forward_ms_2048": round(whole_ms, 3),
        "forward_conv_ms_2048": round(1e3 * fwd_s, 3),
        "roofline": roof,
        "roofline_other": other,
        "conv_layers_ms": {n: round(1e3 * t, 4) for n, t in per.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
