"""Fixed launches of each stepper kernel, for hardware-counter runs.

    python3 -m paper_1901_06535_amd.profile_kernels --workload uniform

runs, on the uniform workload's 16384x16384 grid, a few launches of the
FP32 T-step kernels the benchmark's autotuner may pick (row pipelines, T = 6..9;
LDS tiles), of the FP32 and FP64 one-step kernels and of the FP64 T-step
kernel; ``--workload circuit`` runs every FP32 T-step candidate on the
circuit workload's 4096x4096 grid.  Both end with three 1 GiB launches of the
plain copy kernel (the reading that scales memory counters to bytes).  Under

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1901_06535_amd.profile_kernels --workload W

each dispatch gets its own counter values.  Prints what it launched.

    python3 -m paper_1901_06535_amd.profile_kernels --summarize FETCH.csv WRITE.csv --workload W

turns the two counter runs' CSV files into per-launch HBM bytes: each
kernel's average FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by what
the same counters read for the 1 GiB copy, merged into profiles/traffic.json
under keys naming the kernel and the grid, with the hash of the stepper's
kernel sources, comments and layout aside (readers ignore entries taken on
other code), and printed
as a table;

    python3 -m paper_1901_06535_amd.profile_kernels --stats KERNEL_STATS.csv

prints the top rows of a rocprofv3 --stats kernel table, and

    python3 -m paper_1901_06535_amd.profile_kernels --valu COUNTERS.csv

the VALU instruction counts and busy fraction of one --pmc run of the
counters in VALU_COUNTERS, and ``--valu-active`` the VALU busy fraction by
time of one run of ACTIVE_COUNTERS.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

import numpy as np

from . import inputs, rdc

HERE = os.path.dirname(os.path.abspath(__file__))
STEPPER_SOURCES = ("cell.h", "tile.h", "kernels.h", "kernels.hip", "stream_pipe.h", "stream.hip",
                   "stream64.hip", "tiles_impl.h")


def code_text(src: str) -> str:
    """A source's text with its comments removed and every run of white
    space made one space: what the compiler sees, so that an edit of a
    comment or of the layout does not orphan counters taken on the same
    code."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def source_hash() -> str:
    """Hash of the code (comments and layout aside) of the sources the
    stepper kernels are compiled from, and of their per-source compiler
    flags."""
    from .build import SOURCE_FLAGS
    h = hashlib.sha256()
    for f in STEPPER_SOURCES:
        with open(os.path.join(HERE, "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
        h.update(b"\0")
        h.update(" ".join(SOURCE_FLAGS.get(f, [])).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("rdc::nn::(anonymous namespace)::", "")
    n = n.replace("rdc::(anonymous namespace)::", "")
    m = re.match(r"k_stepT64<(\d+), (\d+), (\w+)>", n)
    if m:
        return "k_stepT64<T=%s,rows=%d%s>" % (m.group(1), 8 * int(m.group(2)),
                                             ",arrival" if m.group(3) == "true" else "")
    m = re.match(r"k_stepT<(\d+), (\d+), (\w+)>", n)
    if m:
        return "k_stepT<T=%s,rows=%d%s>" % (m.group(1), 8 * int(m.group(2)),
                                           ",arrival" if m.group(3) == "true" else "")
    m = re.match(r"k_stream<(\d+)(, \w+)?>", n)
    if m:
        return "k_stream<T=%s>" % m.group(1)
    m = re.match(r"k_stream64<(\d+)(, \w+)?>", n)
    if m:
        return "k_stream64<T=%s>" % m.group(1)
    m = re.match(r"k_step1<(\w+), (\w+)>", n)
    if m:
        return "k_step1<%s%s>" % (m.group(1), ",arrival" if m.group(2) == "true" else "")
    return re.sub(r"\(.*", "", n)


def _counter_means(path: str, counter: str):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in vals.items()}


def stats(path: str, top: int = 20) -> None:
    """Print the top rows of a rocprofv3 --stats kernel table."""
    rows = [(_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]), float(r["Percentage"]))
            for r in csv.DictReader(open(path))]
    for name, calls, avg, pct in rows[:top]:
        print("%-40s calls=%6d avg_us=%9.2f pct=%6.2f" % (name[:40], calls, avg / 1e3, pct))


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_INSTS_LDS", "GRBM_GUI_ACTIVE")


# VALU time: cycles the SIMDs spend executing VALU instructions (quad-cycles,
# so multi-cycle instructions count as long as they run), the FP32
# transcendental instructions among them, and the waves' waiting time.
ACTIVE_COUNTERS = ("SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F32",
                   "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES",
                   "GRBM_GUI_ACTIVE")


def valu_active(path: str, cus: int = 256, xcds: int = 8) -> None:
    """Per-dispatch averages of one rocprofv3 --pmc run of ACTIVE_COUNTERS for
    each stepper kernel: VALU busy by time = SQ_ACTIVE_INST_VALU (quad-cycles
    summed over the SIMDs) / (GRBM_GUI_ACTIVE / xcds * cus), next to the
    issue count's 4-cycle estimate; the quad-cycles beyond one per issued
    instruction, per transcendental instruction; and the fraction of wave
    cycles spent waiting to issue."""
    m = {c: _counter_means(path, c) for c in ACTIVE_COUNTERS}
    for k in sorted(m["SQ_ACTIVE_INST_VALU"]):
        if not k.startswith("k_st") and k != "k_copy16":
            continue
        g = lambda c: m[c].get(k, (float("nan"), 0))[0]
        gui = g("GRBM_GUI_ACTIVE") / xcds * cus
        act, ins, tr = g("SQ_ACTIVE_INST_VALU"), g("SQ_INSTS_VALU"), g("SQ_INSTS_VALU_TRANS_F32")
        # (FP64 kernels' reciprocals are not FP32 transcendentals)
        extra = (act - ins) / tr if tr > 0.01 * ins else float("nan")
        print("%-30s VALU_active=%.4g insts=%.4g trans_f32=%.4g -> VALU busy by time %.1f%% "
              "(issue count x 4 cycles: %.1f%%), extra quad-cycles per transcendental %.2f, "
              "waiting %.0f%% of wave cycles (LDS %.1f%%)"
              % (k, act, ins, tr, 100 * act / gui, 100 * ins / gui, extra,
                 100 * g("SQ_WAIT_INST_ANY") / g("SQ_WAVE_CYCLES"),
                 100 * g("SQ_WAIT_INST_LDS") / g("SQ_WAVE_CYCLES")))


def valu(path: str, cus: int = 256, xcds: int = 8) -> None:
    """Per-dispatch averages of the VALU counters of one rocprofv3 --pmc run
    (VALU_COUNTERS) for each stepper kernel, and the VALU busy fraction: a
    wave64 VALU instruction occupies one SIMD16 for 4 cycles, so busy =
    SQ_INSTS_VALU / (GRBM_GUI_ACTIVE / xcds * cus) (4 SIMDs x 1/4)."""
    m = {c: _counter_means(path, c) for c in VALU_COUNTERS}
    for k in sorted(m["SQ_INSTS_VALU"]):
        if not k.startswith("k_st") and k != "k_copy16":
            continue
        g = lambda c: m[c].get(k, (float("nan"), 0))[0]
        gui = g("GRBM_GUI_ACTIVE")
        busy = g("SQ_INSTS_VALU") / (gui / xcds * cus) if gui > 0 else float("nan")
        print("%-30s VALU_insts=%.4g waves=%.4g busy_cycles=%.4g gui=%.4g lds=%.4g -> VALU busy %.0f%%"
              % (k, g("SQ_INSTS_VALU"), g("SQ_WAVES"), g("SQ_BUSY_CYCLES"), gui,
                 g("SQ_INSTS_LDS"), 100 * busy))


GRIDS = {"uniform": 16384, "circuit": 4096}


def traffic_key(kernel: str, grid: int):
    """profiles/traffic.json key of a kernel (short name) on an n x n grid."""
    m = re.match(r"k_stepT<T=(\d+),rows=(\d+)>$", kernel)
    if m:
        return "stepT_T%s_r%s_%dx%d" % (m.group(1), m.group(2), grid, grid)
    m = re.match(r"k_stream<T=(\d+)>$", kernel)
    if m:
        return "stream_T%s_%dx%d" % (m.group(1), grid, grid)
    m = re.match(r"k_stream64<T=(\d+)>$", kernel)
    if m:
        return "stream64_T%s_%dx%d" % (m.group(1), grid, grid)
    m = re.match(r"k_stepT64<T=(\d+),rows=(\d+)>$", kernel)
    if m:
        return "stepT64_T%s_r%s_%dx%d" % (m.group(1), m.group(2), grid, grid)
    base = {"k_step1<float>": "step1", "k_step1<double>": "step1_f64"}.get(kernel)
    return "%s_%dx%d" % (base, grid, grid) if base else None


def summarize(fetch_csv: str, write_csv: str, out_json: str, workload: str) -> None:
    f = _counter_means(fetch_csv, "FETCH_SIZE")
    w = _counter_means(write_csv, "WRITE_SIZE")
    gib_kib = (1 << 30) / 1024
    sf, sw = gib_kib / f["k_copy16"][0], gib_kib / w["k_copy16"][0]
    try:
        with open(out_json) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        rec = {}
    rec["_note"] = ("Per-launch HBM bytes of each kernel from rocprofv3 FETCH_SIZE and "
                    "WRITE_SIZE (KiB per dispatch), scaled by the readings of a 1 GiB copy "
                    "kernel; source_hash identifies the stepper sources the counters were "
                    "taken on.")
    rec.setdefault("scale", {})[workload] = {"fetch": round(sf, 4), "write": round(sw, 4)}
    print("scale FETCH x%.4f WRITE x%.4f (copy kernel, 1 GiB read + 1 GiB written)" % (sf, sw))
    h = source_hash()
    for k in sorted(f):
        if k not in w or k == "k_copy16" or not k.startswith("k_st"):
            continue
        rd, wr = f[k][0] * 1024 * sf, w[k][0] * 1024 * sw
        key = traffic_key(k, GRIDS[workload])
        print("%-28s n=%2d fetch_KiB=%12.1f write_KiB=%12.1f -> read_MB=%9.1f written_MB=%9.1f"
              % (k, f[k][1], f[k][0], w[k][0], rd / 1e6, wr / 1e6))
        if key:
            rec[key] = {"kernel": k, "bytes_read": int(rd), "bytes_written": int(wr),
                        "bytes_per_launch": int(rd + wr), "source_hash": h}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)


TILE_CANDIDATES = [(T, r) for T in (4, 6, 8, 9, 10, 11, 12) for r in (48, 56, 64, 80)]
STREAM_CANDIDATES = (4, 6, 8, 9, 10, 11, 12)
UNIFORM_TILES = [(8, 56), (8, 64), (10, 64), (11, 64), (12, 64)]
CANDIDATES64 = [(8, 56), (8, 64), (8, 1)]
LAUNCHES = 4


def _launch_all(sim, shapes, log, grid):
    for T, rows in shapes:
        sim.set_block(T)
        sim.set_tile_rows(rows)
        sim.step(LAUNCHES * T)
        name = ("k_stream<T=%d>" % T) if rows == 1 else ("k_stepT<T=%d,rows=%d>" % (T, rows))
        log.append({"kernel": name, "grid": grid, "launches": LAUNCHES})


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="uniform", choices=sorted(GRIDS))
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--stats", metavar="KERNEL_STATS_CSV")
    ap.add_argument("--valu", metavar="COUNTER_CSV")
    ap.add_argument("--valu-active", metavar="COUNTER_CSV")
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(HERE), "profiles",
                                                  "traffic.json"))
    args = ap.parse_args()
    if args.summarize:
        return summarize(args.summarize[0], args.summarize[1], args.out, args.workload)
    if args.stats:
        return stats(args.stats, args.top)
    if args.valu:
        return valu(args.valu)
    if args.valu_active:
        return valu_active(args.valu_active)
    log = []
    n = GRIDS[args.workload]
    if args.workload == "circuit":
        wl = inputs.circuit(n=n, seed=1002, steps=10000, ndisks=256)
    else:
        wl = inputs.uniform_random_phi(n=n, seed=1003, steps=2000)
    sim = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
    sim.set_phi(wl.phi)
    sim.write(wl.u0, wl.v0)
    sim.stimulate([(s.cx, s.cy, s.r) for s in wl.stimuli[:32]])
    grid = [wl.nx, wl.ny]
    stream = [(T, 1) for T in STREAM_CANDIDATES]
    if args.workload == "circuit":
        _launch_all(sim, stream + TILE_CANDIDATES, log, grid)
    else:
        _launch_all(sim, stream + UNIFORM_TILES, log, grid)
        sim.set_block(1)
        sim.step(LAUNCHES)
        log.append({"kernel": "k_step1<float>", "grid": grid, "launches": LAUNCHES})
    sim.synchronize()
    sim.close()

    if args.workload == "uniform":
        # FP64 on the same grid: the one-step kernel and the T-step kernel.
        b64 = rdc.Sim(n, n, wl.params, "fp64")
        b64.set_phi(wl.phi.astype(np.float64))
        b64.set_block(1)
        b64.step(LAUNCHES)
        log.append({"kernel": "k_step1<double>", "grid": grid, "launches": LAUNCHES})
        for T, rows in CANDIDATES64:
            b64.set_block(T)
            b64.set_tile_rows(rows)
            b64.step(LAUNCHES * T)
            log.append({"kernel": ("k_stream64<T=%d>" % T) if rows == 1 else
                        "k_stepT64<T=%d,rows=%d>" % (T, rows), "grid": grid,
                        "launches": LAUNCHES})
        b64.synchronize()
        b64.close()

    nb = 1 << 30
    src = torch.zeros(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        rdc.rdc_copy(dst.data_ptr(), src.data_ptr(), nb, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    log.append({"kernel": "k_copy16", "bytes_read": nb, "bytes_written": nb, "launches": 3})
    print(json.dumps(log), flush=True)


if __name__ == "__main__":
    main()
