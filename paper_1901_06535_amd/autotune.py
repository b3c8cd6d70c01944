"""Autotuner for the stepper's launch shape: steps per launch T and the
layout of the temporal-blocking kernels (LDS tile height, or the
register-resident row pipelines, rows = 1).

Throughput depends on the grid's shape (how its width and height divide into
256-column tiles or strips, how many of them each XCD gets) and on the chip,
not on the data, so a choice is timed once per (GPU architecture, stepper
sources, shape) and cached as JSON.  Timing uses HIP events on the
stream over whole launches of each candidate, after a warm-up launch, on a
scratch grid (or batch) of the same shapes and parameters, so the caller's
state, step index and arrival map are untouched.

Cache: $RDC_AUTOTUNE_CACHE, default ~/.cache/rdc/autotune.json; entries are
keyed "<arch>/<source hash>/<kind>/<shape>".
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

from .profile_kernels import source_hash

DEFAULT_T = (4, 6, 8, 9, 10, 11, 12)
# LDS tile heights, and 1 = the row-pipeline kernel (rdc.RDC_TILE_STREAM)
DEFAULT_ROWS = (48, 56, 64, 80, 1)
# Most steps per launch the row-pipeline kernels take, per precision (FP32:
# 12 on grids whose width is a multiple of 4 and at least 256; on other
# grids such launches run on LDS tiles), and the batched ones.
MAX_T_STREAM = {"fp32": 12, "fp64": 8}
MAX_T_BATCH_STREAM = 11
# Most steps per launch the library's tile kernels take, per precision
# (rdc_set_block; the batched kernels are FP32).
MAX_T = {"fp32": 12, "fp64": 8}


def cache_path() -> str:
    return os.environ.get("RDC_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rdc", "autotune.json"))


def _load() -> Dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: Dict) -> None:
    data = _load()
    data[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                                  # a read-only home only costs re-tuning


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def key_for(kind: str, shape: str) -> str:
    return "%s/%s/%s/%s" % (_arch(), source_hash(), kind, shape)


def _time(step, set_shape, stream, T: int, rows: int, launches: int) -> float:
    """Seconds per Euler step of `launches` launches of (T, rows)."""
    import torch
    set_shape(T, rows)
    step(T)                                   # warm-up launch (code object load, caches)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step(T * launches)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (T * launches)


def _search(step, set_shape, stream, Ts: Iterable[int], rows: Iterable[int],
            launches: int, max_stream: int = MAX_T_STREAM["fp32"]
            ) -> Tuple[Tuple[int, int], Dict[str, float]]:
    table = {}
    for T in Ts:
        for r in rows:
            if r == 1 and T > max_stream:
                continue                      # such launches would run as 56-row tiles
            table["T%d_r%d" % (T, r)] = _time(step, set_shape, stream, T, r, launches)
    best = min(table, key=table.get)
    T, r = (int(x) for x in best[1:].split("_r"))
    return (T, r), table


def tune_sim(sim, Ts: Sequence[int] = DEFAULT_T, rows: Sequence[int] = DEFAULT_ROWS,
             launches: int = 24, use_cache: bool = True) -> Dict:
    """Pick (T, rows) for an `rdc.Sim` (FP32 or FP64), set them on it and
    return {"T", "rows", "us_per_step", "table", "cached"}."""
    from . import rdc
    key = key_for("single" if sim.dtype == "fp32" else "single_" + sim.dtype,
                  "%dx%d" % (sim.nx, sim.ny))
    hit = _load().get(key) if use_cache else None
    if hit:
        rec = dict(hit, cached=True)
    else:
        scratch = rdc.Sim(sim.nx, sim.ny, sim.params, sim.dtype, device=sim.device,
                          stream=sim.stream)
        Ts = [T for T in Ts if T <= MAX_T[sim.dtype]]

        def set_shape(T, r):
            scratch.set_block(T)
            scratch.set_tile_rows(r)
        (T, r), table = _search(scratch.step, set_shape, scratch.stream, Ts, rows, launches,
                                MAX_T_STREAM[sim.dtype])
        scratch.close()
        rec = {"T": T, "rows": r, "us_per_step": round(1e6 * table["T%d_r%d" % (T, r)], 3),
               "table": {k: round(1e6 * v, 3) for k, v in table.items()}}
        _store(key, rec)
        rec = dict(rec, cached=False)
    sim.set_block(rec["T"])
    sim.set_tile_rows(rec["rows"])
    return rec


def tune_batch(batch, Ts: Sequence[int] = DEFAULT_T, rows: Sequence[int] = (48, 56, 64, 1),
               launches: int = 24, use_cache: bool = True) -> Dict:
    """Pick (T, rows) for an `rdc.BatchSim` (keyed by its list of grid sizes
    and its whole-grid path setting, which decides the grids that are
    tiled), set them and return the record."""
    import hashlib
    from . import rdc
    sizes = ",".join("%dx%d" % (nx, ny) for nx, ny, _, _ in batch.shapes)
    res = batch.resident_max_cells
    key = key_for("batch", "%d:%s:res%d" % (len(batch.shapes),
                                            hashlib.sha256(sizes.encode()).hexdigest()[:16], res))
    hit = _load().get(key) if use_cache else None
    if hit:
        rec = dict(hit, cached=True)
    else:
        scratch = rdc.BatchSim(batch.specs, device=batch.device, stream=batch.stream)
        scratch.set_resident(res)             # the same grids tiled as in `batch`
        Ts = [T for T in Ts if T <= MAX_T["fp32"]]
        (T, r), table = _search(scratch.step, scratch.set_block, scratch.stream, Ts, rows,
                                launches, MAX_T_BATCH_STREAM)
        scratch.close()
        rec = {"T": T, "rows": r, "us_per_step": round(1e6 * table["T%d_r%d" % (T, r)], 3),
               "table": {k: round(1e6 * v, 3) for k, v in table.items()}}
        _store(key, rec)
        rec = dict(rec, cached=False)
    batch.set_block(rec["T"], rec["rows"])
    return rec
