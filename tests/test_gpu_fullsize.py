"""Parity at the full workload sizes, on cells the FP64 oracle computed.

The oracle ran each full-size workload once, end to end, and
``tests/golden/make_fullsize_samples.py`` stored its state and arrival times
at a seeded set of sample cells (uniform cells, cells the waves reached, the
domain corners and edges).  Here the GPU runs the same seeded workload:

  * FP64 kernel: u, v and arrival time bit-identical at every sample;
  * FP32, the launch shapes the benchmark's tuner picks from (8 to 12 steps
    per launch; 56- and 64-row tiles): arrival within one cell both ways, and max-abs <= 1e-4 on the
    samples outside the one-cell dilation of the oracle's Euler-unstable set.
"""
import os

import numpy as np
import pytest

from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-4


def _load(name):
    z = np.load(os.path.join(GOLDEN, name + ".npz"), allow_pickle=False)
    return {k: z[k] for k in z.files}


def _workload(name):
    if name == "circuit_4096":
        return inputs.circuit(n=4096, seed=1002, steps=10000, ndisks=256)
    return inputs.uniform_random_phi(n=16384, seed=1003, steps=2000)


def _run(wl, dtype, T=None, rows=None):
    import torch
    s = rdc.Sim(wl.nx, wl.ny, wl.params, dtype)
    s.set_phi(wl.phi)
    s.write(wl.u0, wl.v0)
    if T:
        s.set_block(T)
    if rows:
        s.set_tile_rows(rows)
    s.enable_arrival(0.5)
    s.run_schedule(wl.stimuli, wl.steps)
    s.synchronize()
    return s, torch


def _gather(s, torch, idx):
    u, v = s.current()
    iy = torch.as_tensor(idx[:, 0], device=u.device, dtype=torch.long)
    ix = torch.as_tensor(idx[:, 1], device=u.device, dtype=torch.long)
    arr = s.arrival_plane[:, : s.nx]
    a3 = torch.empty((len(idx), 3, 3), dtype=torch.int32, device=u.device)
    for d in range(3):
        for e in range(3):
            yy = torch.clamp(iy + d - 1, 0, s.ny - 1)
            xx = torch.clamp(ix + e - 1, 0, s.nx - 1)
            a3[:, d, e] = arr[yy, xx]
    return (u[iy, ix].double().cpu().numpy(), v[iy, ix].double().cpu().numpy(),
            a3.cpu().numpy())


@pytest.fixture(scope="module", params=["uniform_16384", "circuit_4096"])
def case(request):
    ref = _load(request.param)
    wl = _workload(request.param)
    assert str(ref["manifest"]) == wl.manifest_json(), "golden file is for another workload"
    assert bool(ref["finite"])
    return request.param, wl, ref


def test_fp64_bitwise_at_samples(case):
    name, wl, ref = case
    print("[case] fp64 %s" % name, flush=True)
    s, torch = _run(wl, "fp64")
    u, v, a3 = _gather(s, torch, ref["idx"])
    s.close()
    assert np.array_equal(u, ref["u"]) and np.array_equal(v, ref["v"])
    assert np.array_equal(a3[:, 1, 1], ref["arr3"][:, 1, 1])


@pytest.mark.parametrize("T,rows", [(8, 56), (8, 64), (10, 64), (11, 64), (12, 56)])
def test_fp32_bench_launch_shape_at_samples(case, T, rows):
    name, wl, ref = case
    print("[case] fp32 %s T=%d rows=%d" % (name, T, rows), flush=True)
    s, torch = _run(wl, "fp32", T=T, rows=rows)
    u, v, a3 = _gather(s, torch, ref["idx"])
    s.close()
    t = a3[:, 1, 1].astype(np.int64)
    r3 = ref["arr3"].reshape(len(t), 9).astype(np.int64)
    g3 = a3.reshape(len(t), 9).astype(np.int64)
    r = ref["arr3"][:, 1, 1].astype(np.int64)
    ok_gpu = (t >= r3.min(1)) & (t <= r3.max(1))
    ok_ref = (r >= g3.min(1)) & (r <= g3.max(1))
    arrived = int((r < np.iinfo(np.int32).max).sum())
    keep = ~ref["masked"]
    du = float(np.abs(u - ref["u"])[keep].max())
    dv = float(np.abs(v - ref["v"])[keep].max())
    print("  samples %d, arrived %d, unmasked %d: arrival violations %d/%d, "
          "max|du| %.3g max|dv| %.3g" % (len(t), arrived, int(keep.sum()),
                                         int((~ok_gpu).sum()), int((~ok_ref).sum()), du, dv))
    assert ok_gpu.all() and ok_ref.all()
    assert arrived > 1000
    assert du <= TOL and dv <= TOL
