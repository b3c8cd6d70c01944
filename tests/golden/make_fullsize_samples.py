"""Writes sampled oracle results for the two full-size workloads:

  circuit_4096.npz   4096x4096 circuit map, 256 input disks, 10,000 steps
  uniform_16384.npz  16384x16384 uniform random phi, 64 disks, 2,000 steps

Each file holds, for a seeded set of sample cells (uniform random cells, cells
the waves reached, the four corners and cells on the domain edges):
  idx        (n, 2) int32  row, column
  u, v       (n,) float64  oracle state at the horizon
  arr3       (n, 3, 3) int32  oracle arrival times (u >= 0.5) over the 3x3
             neighbourhood (edge-clamped), INT32_MAX = never
  masked     (n,) bool    inside the one-cell dilation of the cells the oracle
             ever found Euler-unstable (after step 20)
  first_unstable  int     first such step
and, for the circuit workload, the oracle's whole arrival map:
  arr_bits   np.packbits of the row-major (ny, nx) mask of cells that arrived
  arr_vals   (k,) uint16 their arrival steps in row-major order (all < 65535)
Only the FP64 oracle and the seeded input generators are called.  Runs for a
long time (the 16384^2 case: about half an hour on 8 cores).

    python tests/golden/make_fullsize_samples.py [circuit|uniform]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1901_06535_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def dilate1(m):
    out = m.copy()
    out[1:, :] |= m[:-1, :]
    out[:-1, :] |= m[1:, :]
    o2 = out.copy()
    o2[:, 1:] |= out[:, :-1]
    o2[:, :-1] |= out[:, 1:]
    return o2


def sample_cells(run, rng, n_uniform=2048, n_arrived=2048):
    ny, nx = run.u.shape
    pts = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)]
    for _ in range(64):                                  # domain edges
        pts.append((0, int(rng.integers(0, nx))))
        pts.append((ny - 1, int(rng.integers(0, nx))))
        pts.append((int(rng.integers(0, ny)), 0))
        pts.append((int(rng.integers(0, ny)), nx - 1))
    ys = rng.integers(0, ny, n_uniform)
    xs = rng.integers(0, nx, n_uniform)
    pts += list(zip(ys.tolist(), xs.tolist()))
    ay, ax = np.nonzero(run.arrival < oracle.NEVER)
    if ay.size:
        pick = rng.integers(0, ay.size, n_arrived)
        pts += list(zip(ay[pick].tolist(), ax[pick].tolist()))
    return np.array(sorted(set(pts)), dtype=np.int32)


def write(name, wl, full_arrival=False):
    t0 = time.time()
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params, track_arrival=True, theta=0.5,
                     track_unstable=True, unstable_from=20)
    run.run_schedule(wl.stimuli, wl.steps)
    rng = np.random.default_rng(20260101)
    idx = sample_cells(run, rng)
    ny, nx = run.u.shape
    arr3 = np.empty((len(idx), 3, 3), dtype=np.int32)
    for d in range(3):
        for e in range(3):
            yy = np.clip(idx[:, 0] + d - 1, 0, ny - 1)
            xx = np.clip(idx[:, 1] + e - 1, 0, nx - 1)
            arr3[:, d, e] = run.arrival[yy, xx]
    masked = dilate1(run.unstable.astype(bool))[idx[:, 0], idx[:, 1]]
    extra = {}
    if full_arrival:
        hit = run.arrival < oracle.NEVER
        vals = run.arrival[hit]
        assert vals.max() < 65535
        extra = dict(arr_bits=np.packbits(hit.ravel()), arr_vals=vals.astype(np.uint16))
    np.savez_compressed(os.path.join(HERE, name + ".npz"), idx=idx,
                        u=run.u[idx[:, 0], idx[:, 1]], v=run.v[idx[:, 0], idx[:, 1]],
                        arr3=arr3, masked=masked, first_unstable=np.int64(run.first_unstable),
                        finite=np.bool_(np.isfinite(run.u).all() and np.isfinite(run.v).all()),
                        manifest=np.array(wl.manifest_json()), **extra)
    print(name, "samples", len(idx), "finite", np.isfinite(run.u).all(),
          "arrived", int((run.arrival < oracle.NEVER).sum()), "first_unstable",
          run.first_unstable, "%.0f s" % (time.time() - t0), flush=True)


def main():
    which = sys.argv[1:] or ["circuit", "uniform"]
    if "circuit" in which:
        write("circuit_4096", inputs.circuit(n=4096, seed=1002, steps=10000, ndisks=256),
              full_arrival=True)
    if "uniform" in which:
        write("uniform_16384", inputs.uniform_random_phi(n=16384, seed=1003, steps=2000))


if __name__ == "__main__":
    main()
