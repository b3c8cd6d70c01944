"""Fixed launches of each stepper kernel, for hardware-counter runs.

Runs, on the circuit workload's 4096x4096 grid: a few launches of the
temporal-blocking kernel for every (steps per launch, tile rows) pair the
benchmark's autotuner may pick; on a 16384x16384 grid: a few launches of the
one-step kernel; and three 1 GiB launches of the plain copy kernel (the
reference reading that scales memory counters to bytes).  Under

    rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_1901_06535_amd.profile_kernels

each dispatch gets its own counter values.  Prints what it launched.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import inputs, rdc

CANDIDATES = [(T, r) for T in (4, 6, 8) for r in (48, 56, 64, 80)]
LAUNCHES = 4


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--big", type=int, default=16384)
    args = ap.parse_args()
    log = []
    wl = inputs.circuit(n=args.n, seed=1002, steps=10000, ndisks=256)
    sim = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
    sim.set_phi(wl.phi)
    sim.write(wl.u0, wl.v0)
    sim.stimulate([(s.cx, s.cy, s.r) for s in wl.stimuli[:32]])
    for T, rows in CANDIDATES:
        sim.set_block(T)
        sim.set_tile_rows(rows)
        sim.step(LAUNCHES * T)
        log.append({"kernel": "k_stepT<T=%d,rows=%d>" % (T, rows), "grid": [wl.nx, wl.ny],
                    "launches": LAUNCHES})
    sim.synchronize()
    sim.close()

    n = args.big
    big = rdc.Sim(n, n, inputs.PARAMS_WORKLOAD, "fp32")
    rng = np.random.default_rng(1003)
    big.set_phi((0.04 + 0.04 * rng.random((n, n), dtype=np.float32)).astype(np.float32))
    big.set_block(1)
    big.step(LAUNCHES)
    big.synchronize()
    log.append({"kernel": "k_step1<float>", "grid": [n, n], "launches": LAUNCHES})
    big.close()

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
