"""Parity at the full workload sizes, on cells the FP64 oracle computed.

The oracle ran each full-size workload once, end to end, and
``tests/golden/make_fullsize_samples.py`` stored its state and arrival times
at a seeded set of sample cells (uniform cells, cells the waves reached, the
domain corners and edges).  Here the GPU runs the same seeded workload:

  * FP64 kernel: u, v and arrival time bit-identical at every sample;
  * FP32, the launch shapes the benchmark's tuner picks from (8 to 12 steps
    per launch; 56- and 64-row tiles): arrival within one cell both ways, and max-abs <= 1e-4 on the
    samples outside the one-cell dilation of the oracle's Euler-unstable set;
  * FP32 row pipelines (which take no arrival map): the whole final field
    bit-identical to the tile kernel's.
"""
import os

import numpy as np
import pytest

from metrics import background_far_from_channels

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


def test_fp64_row_pipelines_bitwise_at_samples(case):
    """The FP64 row-pipeline kernel at full size (no arrival map attached, so
    every launch takes it): u and v at the sample cells equal the oracle's."""
    import torch
    name, wl, ref = case
    print("[case] fp64 row pipelines %s T=8" % name, flush=True)
    s = rdc.Sim(wl.nx, wl.ny, wl.params, "fp64")
    s.set_phi(wl.phi.astype(np.float64))
    s.write(wl.u0, wl.v0)
    s.set_block(8)
    s.set_tile_rows(rdc.RDC_TILE_STREAM)
    s.run_schedule(wl.stimuli, wl.steps)
    u, v = s.current()
    iy = torch.as_tensor(ref["idx"][:, 0], device=u.device, dtype=torch.long)
    ix = torch.as_tensor(ref["idx"][:, 1], device=u.device, dtype=torch.long)
    gu, gv = u[iy, ix].cpu().numpy(), v[iy, ix].cpu().numpy()
    s.close()
    assert np.array_equal(gu, ref["u"]) and np.array_equal(gv, ref["v"])


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
    if name == "circuit_4096":
        # sampled cells of the phi = 0.2 background away from the channels:
        # the period-2 orbit, the same phase in both precisions
        p2 = background_far_from_channels(wl.phi)[ref["idx"][:, 0], ref["idx"][:, 1]]
        du2 = float(np.abs(u - ref["u"])[p2].max())
        dv2 = float(np.abs(v - ref["v"])[p2].max())
        print("  period-2 background samples %d: max|du| %.3g max|dv| %.3g"
              % (int(p2.sum()), du2, dv2))
        assert p2.sum() > 1000
        assert du2 <= TOL and dv2 <= TOL


def _oracle_arrival(ref, ny, nx):
    hit = np.unpackbits(ref["arr_bits"], count=ny * nx).astype(bool).reshape(ny, nx)
    arr = np.full((ny, nx), np.iinfo(np.int32).max, dtype=np.int64)
    arr[hit] = ref["arr_vals"]
    return arr


def _neigh_minmax_gpu(torch, a):
    """Min and max over each cell's 3x3 neighbourhood (edge cells repeat the
    edge), on the GPU; arrival times as float64 (exact)."""
    t = a.to(torch.float64)[None, None]
    p = torch.nn.functional.pad(t, (1, 1, 1, 1), mode="replicate")
    hi = torch.nn.functional.max_pool2d(p, 3, stride=1)[0, 0]
    lo = -torch.nn.functional.max_pool2d(-p, 3, stride=1)[0, 0]
    return lo, hi


@pytest.mark.parametrize("dtype,T,rows", [("fp64", 8, 56), ("fp32", 8, 64), ("fp32", 11, 64)])
def test_circuit_arrival_over_the_whole_field(dtype, T, rows):
    """The 4096^2 circuit run's arrival map (first step with u >= 0.5) in
    every cell against the oracle's whole map: FP64 identical, FP32 within
    one cell both ways."""
    import torch
    ref = _load("circuit_4096")
    wl = _workload("circuit_4096")
    assert str(ref["manifest"]) == wl.manifest_json(), "golden file is for another workload"
    print("[case] whole-field arrival %s T=%d rows=%d" % (dtype, T, rows), flush=True)
    oracle_arr = _oracle_arrival(ref, wl.ny, wl.nx)
    s, _ = _run(wl, dtype, T=T, rows=rows)
    gpu = s.arrival_plane[:, : s.nx].to(torch.int64)
    s.close()
    ref_t = torch.as_tensor(oracle_arr, device=gpu.device)
    if dtype == "fp64":
        assert torch.equal(gpu, ref_t)
        return
    lo, hi = _neigh_minmax_gpu(torch, ref_t)
    g = gpu.to(torch.float64)
    bad_gpu = int(((g < lo) | (g > hi)).sum())
    lo2, hi2 = _neigh_minmax_gpu(torch, gpu)
    r = ref_t.to(torch.float64)
    bad_ref = int(((r < lo2) | (r > hi2)).sum())
    arrived = int((ref_t < np.iinfo(np.int32).max).sum())
    print("  arrived %d of %d cells; violations %d / %d" % (arrived, wl.nx * wl.ny, bad_gpu,
                                                          bad_ref))
    assert arrived > 500000
    assert bad_gpu == 0 and bad_ref == 0


@pytest.mark.parametrize("T", [9, 11, 12])
def test_fp32_row_pipelines_equal_tiles_over_the_whole_field(case, T):
    name, wl, ref = case
    print("[case] fp32 row pipelines %s T=%d" % (name, T), flush=True)
    out = []
    for t, rows in ((8, 64), (T, rdc.RDC_TILE_STREAM)):
        s = rdc.Sim(wl.nx, wl.ny, wl.params, "fp32")
        s.set_phi(wl.phi)
        s.write(wl.u0, wl.v0)
        s.set_block(t)
        s.set_tile_rows(rows)
        s.run_schedule(wl.stimuli, wl.steps)
        u, v = s.current()
        out.append((u.clone(), v.clone()))
        s.close()
    import torch
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
