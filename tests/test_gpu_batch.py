"""Batched simulations on the GPU: every grid of a batch evolves bit-identically
to the same grid stepped alone (same per-cell expression), whether it runs
tiled or whole in LDS (the small grids' path), graph replays equal eager
stepping, and batched grids match the FP64 oracle."""
import numpy as np
import pytest

import oracle
from metrics import masked_maxabs
from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (5, 300), (300, 7), (64, 64), (200, 333), (257, 129), (241, 17), (96, 500),
         (33, 65), (128, 256), (400, 41), (17, 17)]


def _case(seed=7):
    rng = np.random.default_rng(seed)
    specs, states, disks = [], [], []
    for i, (nx, ny) in enumerate(SIZES):
        p = dict(inputs.PARAMS_WORKLOAD)
        p["eps"] = float(rng.uniform(0.02, 0.03))
        u, v, phi = inputs.random_state(nx, ny, seed=100 + i, umax=0.02, vmax=0.02)
        specs.append((nx, ny, p))
        states.append((u, v, phi))
        disks.append((i, nx // 2, ny // 2, 3))
    return specs, states, disks


def _batch(specs, states, disks, T, rows=56):
    b = rdc.BatchSim(specs)
    for i, (u, v, phi) in enumerate(states):
        b.set_phi(i, phi)
        b.write(i, u, v)
    b.set_block(T, rows)
    b.stimulate(disks)
    return b


def _single(spec, state, disk, T, nsteps):
    nx, ny, p = spec
    u, v, phi = state
    s = rdc.Sim(nx, ny, p, "fp32")
    s.set_phi(phi)
    s.write(u, v)
    s.set_block(T)
    s.stimulate([disk[1:]])
    s.step(nsteps)
    out = s.read()
    s.close()
    return out


STREAM = rdc.RDC_TILE_STREAM


@pytest.mark.parametrize("T,rows", [(8, 56), (5, 48), (8, 64), (1, 56), (12, 48), (10, 64),
                                    (8, STREAM), (11, STREAM), (3, STREAM), (1, STREAM)])
def test_batch_equals_single_grids_bitwise(T, rows):
    specs, states, disks = _case()
    b = _batch(specs, states, disks, T, rows)
    b.step(37)
    for i in range(len(specs)):
        got = b.read(i)
        ref = _single(specs[i], states[i], disks[i], 1, 37)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (i, SIZES[i])
    b.close()


@pytest.mark.parametrize("T", [2, 5, 8, 11])
def test_batch_row_pipelines_on_every_grid_bitwise(T):
    """The whole-grid path off, so every grid of the batch (1 x 1, 5 x 300,
    17 x 17 up to 200 x 333) runs on the batched row pipelines: one wave per
    (grid, strip, segment), segments planned over all grids; launches of
    exactly T steps and a shorter one; every grid bit-identical to the one-
    step kernel on it alone."""
    specs, states, disks = _case(seed=13)
    b = _batch(specs, states, disks, T, STREAM)
    b.set_resident(0)
    assert b.resident_count() == 0
    n = 3 * T + (T - 1 if T > 2 else 0)
    b.step(n)
    for i in range(len(specs)):
        got = b.read(i)
        ref = _single(specs[i], states[i], disks[i], 1, n)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (i, SIZES[i])
    b.close()


@pytest.mark.parametrize("T", [8, 11])
def test_batch_row_pipelines_in_several_rounds_bitwise(T):
    """600 grids of 300 x 200 and 257 x 190 (two strips each): one round of
    resident waves would leave every grid a single 200-row segment, so the
    plan cuts them into 40-row segments, 6,000 items in three rounds of
    waves, longest first.  Every grid bit-identical to the same batch
    stepped one step per launch on tiles."""
    specs, states = [], []
    rng = np.random.default_rng(21)
    for i in range(600):
        nx, ny = (300, 200) if i % 2 == 0 else (257, 190)
        p = dict(inputs.PARAMS_WORKLOAD)
        p["eps"] = float(rng.uniform(0.024, 0.03))
        specs.append((nx, ny, p))
        states.append(inputs.random_state(nx, ny, seed=500 + i, umax=0.02, vmax=0.02))
    disks = [(i, specs[i][0] // 2, specs[i][1] // 3, 4) for i in range(0, 600, 7)]
    runs = []
    for shape in ((T, STREAM), (1, 56)):
        print("[case] batch of 600, T=%d rows=%d" % shape, flush=True)
        b = _batch(specs, states, disks, *shape)
        b.set_resident(0)
        b.step(3 * T - 1)
        runs.append([b.read(i) for i in range(len(specs))])
        b.close()
    for i, (a, c) in enumerate(zip(*runs)):
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), i


def test_batch_row_pipeline_graph_replays_equal_eager_steps():
    specs, states, disks = _case(seed=15)
    eager = _batch(specs, states, disks, 10, STREAM)
    graph_b = _batch(specs, states, disks, 10, STREAM)
    for x in (eager, graph_b):
        x.set_resident(0)
    g = graph_b.capture(40)          # 4 launches of 10
    for rep in range(3):
        eager.step(40)
        g.launch()
        graph_b.synchronize()
        for i in range(len(specs)):
            a = eager.read(i)
            c = graph_b.read(i)
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), (rep, i)
    g.close()
    eager.close()
    graph_b.close()


def test_batch_graph_replays_equal_eager_steps():
    specs, states, disks = _case(seed=9)
    eager = _batch(specs, states, disks, 8)
    graph_b = _batch(specs, states, disks, 8)
    g = graph_b.capture(24)          # 3 launches of 8 -> recorded as an even count
    for rep in range(3):
        eager.step(24)
        g.launch()
        graph_b.synchronize()
        for i in (0, 4, 7, 11):      # eager work between replays
            a = eager.read(i)
            c = graph_b.read(i)
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), (rep, i)
    g.close()
    eager.close()
    graph_b.close()


def test_batch_graph_replay_after_eager_steps_of_odd_launch_count():
    """Eager steps of an odd number of launches between replays leave the
    state in the other ping-pong copy; the replay starts from it anyway."""
    specs, states, disks = _case(seed=11)
    eager = _batch(specs, states, disks, 8)
    graph_b = _batch(specs, states, disks, 8)
    g = graph_b.capture(16)
    for n_eager in (8, 5, 16, 3):     # 1, 1, 2 and 1 launches of T <= 8
        eager.step(n_eager)
        graph_b.step(n_eager)
        eager.step(16)
        g.launch()
        graph_b.synchronize()
        for i in range(len(specs)):
            a = eager.read(i)
            c = graph_b.read(i)
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), (n_eager, i)
    assert graph_b.step_index == eager.step_index
    g.close()
    eager.close()
    graph_b.close()


def test_batch_matches_oracle_per_grid():
    specs, states, disks = _case(seed=3)
    b = _batch(specs, states, disks, 8)
    b.step(120)
    for i in (1, 4, 7, 10):
        nx, ny, p = specs[i]
        u, v, phi = states[i]
        run = oracle.Run(u, v, phi, p)
        run.stimulate([disks[i][1:]])
        run.advance(120)
        gu, gv = b.read(i)
        assert masked_maxabs(gu, run.u) <= 1e-4 and masked_maxabs(gv, run.v) <= 1e-4, i
    b.close()


@pytest.mark.parametrize("path", ["whole_grid", "tiles", "row_pipelines"])
def test_batch_nonfinite_flag_is_per_grid(path):
    """u = -q planted in one cell of grid 1 makes (u - q)/(u + q) infinite:
    only grid 1's flag is raised, on each path the grids can take."""
    specs, states, disks = _case(seed=4)
    b = rdc.BatchSim(specs[:3])
    if path != "whole_grid":
        b.set_resident(0)
        b.set_block(8, 56 if path == "tiles" else STREAM)
    for i in range(3):
        b.set_phi(i, states[i][2])
        b.write(i, states[i][0], states[i][1])
    bad = states[1][0].copy()
    bad.flat[bad.size // 2] = -inputs.PARAMS_WORKLOAD["q"]   # u + q == 0
    b.write(1, bad, states[1][1])
    b.step(16)
    b.read(0)
    b.read(2)
    with pytest.raises(rdc.RdcError) as e:
        b.read(1)
    assert e.value.status == rdc.RDC_E_NONFINITE
    b.close()


def test_sweep_workload_stability_matches_the_oracle():
    """A slice of the 512-grid sweep (own eps, phi_excitable, channel lattice
    on phi=0.2, disks inside channels).  Forward Euler at dt=0.001 diverges in
    the refractory tails of the stiffest grids (eps near 0.02) -- the FP64
    oracle does too.  Grids with eps >= 0.025 stay finite for 2,000 steps with
    waves travelling; grids the library flags non-finite are stiff ones, and
    the oracle diverges on the smallest of them as well."""
    sims, _ = inputs.batch_sweep(count=48, seed=1004)
    b = rdc.BatchSim([(s.nx, s.ny, s.params) for s in sims])
    for i, s in enumerate(sims):
        b.set_phi(i, s.phi)
    b.stimulate([(i, d.cx, d.cy, d.r) for i, s in enumerate(sims) for d in s.stimuli])
    b.step(2000)
    vmax, flagged = 0.0, []
    for i, s in enumerate(sims):
        try:
            u, v = b.read(i)
            assert np.isfinite(u).all() and np.isfinite(v).all()
            vmax = max(vmax, float(v.max()))
        except rdc.RdcError as e:
            assert e.status == rdc.RDC_E_NONFINITE
            flagged.append(i)
    b.close()
    print("  flagged non-finite: %s" % [(i, round(sims[i].params["eps"], 4)) for i in flagged])
    assert vmax > 0.05
    assert all(sims[i].params["eps"] < 0.025 for i in flagged)
    if flagged:
        i = min(flagged, key=lambda j: sims[j].nx * sims[j].ny)
        s = sims[i]
        run = oracle.Run(np.zeros((s.ny, s.nx)), np.zeros((s.ny, s.nx)), s.phi, s.params)
        run.stimulate([(d.cx, d.cy, d.r) for d in s.stimuli])
        run.advance(2000)
        assert not (np.isfinite(run.u).all() and np.isfinite(run.v).all())


# ---------------------------------------------------------------- whole-grid LDS path

# Shapes of the whole-grid kernel's layouts: one column per thread with 1..16
# rows, full and ragged last row groups, single rows and columns, the widest
# (1024 columns) and the largest (128 x 128) grids; the last one is tiled.
RES_SIZES = [(1, 7), (7, 1), (2, 3000), (1000, 10), (1024, 16), (128, 128), (37, 199),
             (333, 41), (100, 70), (16, 16), (300, 200)]


def _res_case(seed):
    rng = np.random.default_rng(seed)
    specs, states, disks = [], [], []
    for i, (nx, ny) in enumerate(RES_SIZES):
        p = dict(inputs.PARAMS_WORKLOAD)
        p["eps"] = float(rng.uniform(0.022, 0.03))
        u, v, phi = inputs.random_state(nx, ny, seed=300 + i, umax=0.02, vmax=0.02)
        specs.append((nx, ny, p))
        states.append((u, v, phi))
        disks.append((i, nx // 3, ny // 2, 4))
    return specs, states, disks


@pytest.mark.parametrize("n,T", [(37, 8), (45, 8), (12, 12)])
def test_resident_layouts_equal_single_grids_bitwise(n, T):
    """n steps with T = 8 take 5 (odd: the whole-grid launches write the
    other ping-pong copy) or 6 tile launches; 12 at T = 12 one."""
    specs, states, disks = _res_case(seed=21)
    b = _batch(specs, states, disks, T)
    assert b.resident_count() == len(RES_SIZES) - 1
    print("[case] resident layouts n=%d T=%d" % (n, T), flush=True)
    b.step(n)
    for i in range(len(specs)):
        got = b.read(i)
        ref = _single(specs[i], states[i], disks[i], 8, n)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (i, RES_SIZES[i])
    b.close()


def test_resident_path_equals_tiled_path_bitwise():
    specs, states, disks = _case(seed=13)
    res = _batch(specs, states, disks, 8)
    tiled = _batch(specs, states, disks, 8)
    tiled.set_resident(0)
    small = sum(nx * ny <= rdc.RDC_BATCH_RESIDENT_DEFAULT for nx, ny, _ in specs)
    assert res.resident_count() == small and tiled.resident_count() == 0
    for n in (19, 8, 40):
        res.step(n)
        tiled.step(n)
        for i in range(len(specs)):
            a, c = res.read(i), tiled.read(i)
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), (n, i)
    res.close()
    tiled.close()


def test_resident_long_call_is_split_and_bitwise():
    """40,000 steps in one call: three whole-grid launches (16,384 steps at
    most each) on an all-small batch."""
    specs, states, disks = _res_case(seed=22)
    pick = [9, 8]                                   # 16 x 16 and 100 x 70
    specs = [specs[i] for i in pick]
    states = [states[i] for i in pick]
    disks = [(j,) + disks[i][1:] for j, i in enumerate(pick)]
    b = _batch(specs, states, disks, 8)
    assert b.resident_count() == 2
    b.step(40000)
    for j in range(2):
        got = b.read(j)
        ref = _single(specs[j], states[j], disks[j], 12, 40000)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), j
    b.close()


def test_resident_graph_and_replan():
    """A graph recorded with whole-grid launches replays like eager steps;
    after rdc_batch_set_resident the old recording is refused."""
    specs, states, disks = _res_case(seed=23)
    eager = _batch(specs, states, disks, 8)
    graph_b = _batch(specs, states, disks, 8)
    g = graph_b.capture(40)
    for rep in range(2):
        eager.step(40)
        g.launch()
        for i in range(len(specs)):
            a, c = eager.read(i), graph_b.read(i)
            assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]), (rep, i)
    graph_b.set_resident(4096)
    with pytest.raises(rdc.RdcError) as e:
        g.launch()
    assert e.value.status == rdc.RDC_E_STATE
    g.close()
    eager.close()
    graph_b.close()
