"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (floating point, the oracle is FP64):
  * FP64 kernels: bit-identical to the oracle, every horizon;
  * FP32 kernels: max-abs <= 1e-4 on the whole field up to the oracle's first
    Euler-unstable step n*, max-abs <= 1e-4 outside the one-cell dilation of
    the cells the oracle ever flags unstable at the horizon, and arrival times
    (first step with u >= 0.5) equal to within one cell;
  * every FP32 launch shape (steps per launch, tile height) bit-identical to
    the one-step kernel.
"""
import numpy as np
import pytest

import oracle
from metrics import (arrival_within_one_cell, arrival_violations, background_far_from_channels,
                     dilate, masked_maxabs)
from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu

TOL = 1e-4


def make_sim(wl, dtype="fp32", T=None, rows=None, arrival=False, theta=0.5):
    s = rdc.Sim(wl.nx, wl.ny, wl.params, dtype)
    s.set_phi(wl.phi)
    s.write(wl.u0, wl.v0)
    if T is not None:
        s.set_block(T)
    if rows:
        s.set_tile_rows(rows)
    if arrival:
        s.enable_arrival(theta)
    return s


def print_case(msg):
    print("[case] " + msg, flush=True)


# ------------------------------------------------------------------ single disk, 256^2

@pytest.fixture(scope="module")
def disk_oracle():
    wl = inputs.single_disk()
    ref = {}
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params, track_arrival=True, track_unstable=True)
    for n in (1, 50, 200, 300, 1000):
        run.run_schedule(wl.stimuli, n)
        ref[n] = (run.u.copy(), run.v.copy(), run.arrival.copy())
    return wl, ref, run.first_unstable, run.unstable.astype(bool)


def test_fp64_single_disk_bitwise(disk_oracle):
    wl, ref, _, _ = disk_oracle
    print_case("fp64 single disk 256^2")
    s = make_sim(wl, "fp64", arrival=True)
    for n in sorted(ref):
        s.run_schedule(wl.stimuli, n)
        u, v = s.read()
        assert np.array_equal(u, ref[n][0]), n
        assert np.array_equal(v, ref[n][1]), n
        assert np.array_equal(s.arrival(), ref[n][2]), n
    s.close()


@pytest.mark.parametrize("T", [1, 8])
def test_fp32_single_disk_masked_parity(disk_oracle, T):
    wl, ref, nstar, unstable = disk_oracle
    print_case("fp32 single disk 256^2 T=%d n*=%d" % (T, nstar))
    assert 200 < nstar < 1000
    s = make_sim(wl, "fp32", T=T, arrival=True)
    # (i) full field up to n*
    for n in (1, 50, 200, 300):
        if n > nstar:
            continue
        s.run_schedule(wl.stimuli, n)
        u, v = s.read()
        assert masked_maxabs(u, ref[n][0]) <= TOL, n
        assert masked_maxabs(v, ref[n][1]) <= TOL, n
    # (ii) at the horizon, outside the one-cell dilation of the unstable set
    s.run_schedule(wl.stimuli, 1000)
    u, v = s.read()
    mask = dilate(unstable, 1)
    du = masked_maxabs(u, ref[1000][0], mask)
    dv = masked_maxabs(v, ref[1000][1], mask)
    full = masked_maxabs(u, ref[1000][0])
    print("  masked max|du|=%.3g max|dv|=%.3g (unmasked %.3g, masked cells %d)"
          % (du, dv, full, int(mask.sum())))
    assert du <= TOL and dv <= TOL
    assert mask.sum() < 0.1 * mask.size
    # (iii) arrival within one cell
    assert arrival_within_one_cell(s.arrival(), ref[1000][2])
    s.close()


# ------------------------------------------------------------------ launch-shape invariance

def _ragged_case(nx=333, ny=275, seed=12):
    u, v, phi = inputs.random_state(nx, ny, seed=seed, umax=0.02, vmax=0.02, phi_lo=0.04,
                                    phi_hi=0.09)
    disks = inputs.random_disks(nx, ny, 12, seed=seed + 1, rmax=7)
    return u, v, phi, [(d.cx, d.cy, d.r) for d in disks]


def _run_fp32(u, v, phi, disks, T, rows, nsteps=(23, 14), params=inputs.PARAMS_WORKLOAD,
              dtype="fp32"):
    ny, nx = u.shape
    s = rdc.Sim(nx, ny, params, dtype)
    s.set_phi(phi)
    s.write(u, v)
    s.set_block(T)
    if rows:
        s.set_tile_rows(rows)
    s.stimulate(disks)
    s.step(nsteps[0])
    s.stimulate(disks[:3])
    s.step(nsteps[1])
    out = s.read()
    s.close()
    return out


def test_every_launch_shape_is_bitwise_equal_to_one_step_kernel():
    u, v, phi, disks = _ragged_case()
    ref = _run_fp32(u, v, phi, disks, T=1, rows=0)
    assert np.isfinite(ref[0]).all()
    for rows in (48, 56, 64, 80, rdc.RDC_TILE_STREAM):
        for T in range(2, 13):
            print_case("T=%d rows=%d" % (T, rows))
            got = _run_fp32(u, v, phi, disks, T=T, rows=rows)
            assert np.array_equal(got[0], ref[0]), (T, rows)
            assert np.array_equal(got[1], ref[1]), (T, rows)


SHAPES = [(1, 1), (1, 7), (7, 1), (2, 2), (8, 8), (3, 300), (300, 3), (65, 63), (257, 129),
          (241, 17)]


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_small_and_ragged_grids_fp64_bitwise(ny, nx):
    u, v, phi = inputs.random_state(nx, ny, seed=nx * 1000 + ny, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 2), (0, 0, 1)]
    run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
    run.stimulate(disks)
    run.advance(60)
    for T, rows in ((1, 0), (3, 48), (8, 48), (8, 80)):
        print_case("fp64 %dx%d T=%d rows=%d" % (ny, nx, T, rows))
        s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, "fp64")
        s.set_phi(phi)
        s.write(u, v)
        s.set_block(T)
        s.set_tile_rows(rows)
        s.stimulate(disks)
        s.step(60)
        gu, gv = s.read()
        s.close()
        assert np.array_equal(gu, run.u) and np.array_equal(gv, run.v), (T, rows)


def test_every_fp64_launch_shape_is_bitwise_equal_to_the_oracle():
    u, v, phi, disks = _ragged_case()
    ny, nx = u.shape
    run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
    run.stimulate(disks)
    run.advance(23)
    run.stimulate(disks[:3])
    run.advance(14)
    for rows in (48, 56, 64, 80, rdc.RDC_TILE_STREAM):
        for T in range(2, 9):
            print_case("fp64 T=%d rows=%d" % (T, rows))
            s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, "fp64")
            s.set_phi(phi)
            s.write(u, v)
            s.set_block(T)
            s.set_tile_rows(rows)
            s.stimulate(disks)
            s.step(23)
            s.stimulate(disks[:3])
            s.step(14)
            gu, gv = s.read()
            s.close()
            assert np.array_equal(gu, run.u) and np.array_equal(gv, run.v), (T, rows)


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_small_and_ragged_grids_fp32_launch_shapes(ny, nx):
    print_case("fp32 shapes %dx%d" % (ny, nx))
    u, v, phi = inputs.random_state(nx, ny, seed=nx * 1000 + ny, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 2)]
    ref = _run_fp32(u, v, phi, disks, T=1, rows=0, nsteps=(20, 19))
    run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
    run.stimulate(disks)
    run.advance(20)
    run.stimulate(disks[:3])
    run.advance(19)
    assert masked_maxabs(ref[0], run.u) <= TOL
    for T, rows in ((3, 48), (8, 48), (3, rdc.RDC_TILE_STREAM), (8, rdc.RDC_TILE_STREAM),
                    (11, rdc.RDC_TILE_STREAM), (12, rdc.RDC_TILE_STREAM)):
        got = _run_fp32(u, v, phi, disks, T=T, rows=rows, nsteps=(20, 19))
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (T, rows)


@pytest.mark.parametrize("ny,nx", [(700, 1000), (97, 1210), (1500, 250), (2049, 515),
                                   (333, 1028), (97, 256)])
def test_row_pipelines_across_strips_and_segments_bitwise(ny, nx):
    """The row-pipeline kernel on grids of several 256-column strips (inner
    strips with 16-byte accesses; edge strips cell by cell, or, for widths
    that are multiples of 4 from 256 on, by mirrored 16-byte blocks; a ragged
    last strip) and many row segments: bit-identical to the one-step kernel
    for every T it takes."""
    u, v, phi = inputs.random_state(nx, ny, seed=nx + 7 * ny, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 4), (3, 5, 3), (nx - 2, ny - 3, 5), (nx // 3, 1, 2)]
    ref = _run_fp32(u, v, phi, disks, T=1, rows=0, nsteps=(25, 18))
    assert np.isfinite(ref[0]).all()
    for T in range(2, 13):          # T = 12 on widths a multiple of 4 (>= 256), else tiles
        print_case("stream %dx%d T=%d" % (ny, nx, T))
        got = _run_fp32(u, v, phi, disks, T=T, rows=rdc.RDC_TILE_STREAM, nsteps=(25, 18))
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), T


@pytest.mark.parametrize("nx", [14848, 14846])
def test_row_pipelines_on_tall_segments_bitwise(nx):
    """Grids of 60-64 strips and 1024 rows: with a wave per (strip, segment)
    and 2048 resident waves, segments are 31-32 rows tall, so a wave walks
    the ramp bodies (where levels with no row yet are left out), whole loop
    bodies and a partial last one (at T = 2..4 the last segment is a single
    row: the ramp bodies only).  Each launch is exactly T steps; bit-identical
    to the one-step kernel for T = 2..12, width a multiple of 4 (mirrored
    16-byte edge blocks) and not (edge strips cell by cell; there T = 12
    runs on the LDS tiles)."""
    ny = 1024
    u, v, phi = inputs.random_state(nx, ny, seed=nx + 3, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 4), (3, 5, 3), (nx - 2, ny - 3, 5), (nx // 3, 1, 2),
             (250, 30, 6), (nx - 300, 40, 6)]
    for T in range(2, 13):
        print_case("stream tall segments %dx%d T=%d" % (ny, nx, T))
        ref = _run_fp32(u, v, phi, disks, T=1, rows=0, nsteps=(2 * T, T))
        assert np.isfinite(ref[0]).all()
        got = _run_fp32(u, v, phi, disks, T=T, rows=rdc.RDC_TILE_STREAM, nsteps=(2 * T, T))
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), T


def test_fp64_row_pipelines_on_tall_segments_equal_the_oracle():
    """The FP64 row pipelines (128-column strips) on 1024 x 7424: 60-67
    strips, segments 31-35 rows tall, so waves walk the ramp bodies, whole
    loop bodies and a partial last one; each launch exactly T steps;
    bit-identical to the oracle for T = 2..8."""
    ny, nx = 1024, 7424
    u, v, phi = inputs.random_state(nx, ny, seed=77, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 4), (3, 5, 3), (nx - 2, ny - 3, 5), (nx // 3, 1, 2)]
    for T in range(2, 9):
        print_case("fp64 stream tall segments %dx%d T=%d" % (ny, nx, T))
        run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
        run.stimulate(disks)
        run.advance(2 * T)
        run.stimulate(disks[:3])
        run.advance(T)
        got = _run_fp32(u, v, phi, disks, T=T, rows=rdc.RDC_TILE_STREAM, nsteps=(2 * T, T),
                        dtype="fp64")
        assert np.array_equal(got[0], run.u) and np.array_equal(got[1], run.v), T


@pytest.mark.parametrize("ny,nx", [(700, 1000), (97, 610), (1500, 250), (2049, 515)])
def test_fp64_row_pipelines_across_strips_and_segments_equal_the_oracle(ny, nx):
    """The FP64 row-pipeline kernel (128-column strips) on grids of several
    strips and many row segments: bit-identical to the oracle for every T it
    takes."""
    u, v, phi = inputs.random_state(nx, ny, seed=nx + 5 * ny, umax=0.02, vmax=0.02)
    disks = [(nx // 2, ny // 2, 4), (3, 5, 3), (nx - 2, ny - 3, 5), (nx // 3, 1, 2)]
    run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
    run.stimulate(disks)
    run.advance(25)
    run.stimulate(disks[:3])
    run.advance(18)
    assert np.isfinite(run.u).all()
    for T in range(2, 9):
        print_case("fp64 stream %dx%d T=%d" % (ny, nx, T))
        got = _run_fp32(u, v, phi, disks, T=T, rows=rdc.RDC_TILE_STREAM, nsteps=(25, 18),
                        dtype="fp64")
        assert np.array_equal(got[0], run.u) and np.array_equal(got[1], run.v), T


# ------------------------------------------------------------------ stimulation, flags, resume

def test_stimulation_matches_oracle_at_edges():
    nx, ny = 70, 45
    u, v, phi = inputs.random_state(nx, ny, seed=2, umax=0.5)
    disks = [(0, 0, 5), (69, 44, 7), (35, 0, 0), (-3, 20, 4), (72, 10, 3), (30, 22, 9)]
    ou = u.astype(np.float64)
    oracle.stimulate(ou, disks)
    s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, "fp64")
    s.set_phi(phi)
    s.write(u, v)
    s.stimulate(disks)
    gu, gv = s.read()
    assert np.array_equal(gu, ou)
    assert np.array_equal(gv, v.astype(np.float64))
    with pytest.raises(rdc.RdcError) as e:
        s.stimulate([(100, 100, 3)])
    assert e.value.status == rdc.RDC_E_INVAL
    s.close()


@pytest.mark.parametrize("dtype,T,rows", [("fp32", 1, 0), ("fp32", 8, 0), ("fp64", 1, 0),
                                          ("fp32", 8, rdc.RDC_TILE_STREAM),
                                          ("fp32", 11, rdc.RDC_TILE_STREAM),
                                          ("fp64", 8, rdc.RDC_TILE_STREAM)])
def test_nonfinite_flag_is_raised_and_cleared(dtype, T, rows):
    nx = ny = 40
    q = inputs.PARAMS_WORKLOAD["q"]
    u = np.zeros((ny, nx), np.float32)
    v = np.zeros((ny, nx), np.float32)
    u[20, 20] = -q          # u + q == 0: the reaction's quotient divides by zero
    s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, dtype)
    s.set_phi(np.full((ny, nx), 0.054, np.float32))
    s.set_block(T)
    if rows:
        s.set_tile_rows(rows)
    s.write(u, v)
    s.step(16)
    _, _ = s.read(allow_nonfinite=True)
    with pytest.raises(rdc.RdcError) as e:
        s.read()
    assert e.value.status == rdc.RDC_E_NONFINITE
    # the zero-copy view reports the flag too, and still gives the planes
    with pytest.raises(rdc.RdcError) as e:
        s.current()
    assert e.value.status == rdc.RDC_E_NONFINITE
    cu, _ = s.current(allow_nonfinite=True)
    assert not np.isfinite(cu.cpu().numpy()).all()
    s.write(np.zeros_like(u), v)
    s.step(16)
    s.read()   # flag cleared by the fresh state
    s.current()
    s.close()


def test_split_run_resume_and_repeat_are_bitwise():
    u, v, phi, disks = _ragged_case(nx=300, ny=200, seed=3)
    def run(splits):
        s = rdc.Sim(300, 200, inputs.PARAMS_WORKLOAD, "fp32")
        s.set_phi(phi)
        s.write(u, v)
        s.set_block(8)
        s.stimulate(disks)
        for n in splits:
            s.step(n)
            a, b = s.read()
            s.write(a, b)       # checkpoint / resume through host memory
        out = s.read()
        s.close()
        return out
    a = run([200])
    b = run([77, 123])
    c = run([200])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


@pytest.mark.parametrize("T,rows", [(8, 0), (11, rdc.RDC_TILE_STREAM), (12, rdc.RDC_TILE_STREAM)])
@pytest.mark.parametrize("sym", ["xflip", "yflip", "transpose"])
def test_fp32_d4_symmetry_is_bitwise(sym, T, rows):
    """A symmetric phi map and stimuli give a bitwise symmetric field, on the
    LDS tiles and on the row pipelines (300 columns: edge strips of mirrored
    16-byte blocks)."""
    n = 300
    _, _, phi = inputs.random_state(n, n, seed=8)
    half = n // 2
    if sym == "xflip":
        phi = np.concatenate([phi[:, :half], phi[:, :half][:, ::-1]], axis=1)
        disks = [(40, 90, 5), (n - 41, 90, 5)]
    elif sym == "yflip":
        phi = np.concatenate([phi[:half], phi[:half][::-1]], axis=0)
        disks = [(90, 40, 5), (90, n - 41, 5)]
    else:
        phi = np.triu(phi) + np.triu(phi, 1).T
        disks = [(40, 200, 5), (200, 40, 5), (100, 100, 4)]
    s = rdc.Sim(n, n, inputs.PARAMS_WORKLOAD, "fp32")
    s.set_phi(np.ascontiguousarray(phi))
    s.write(np.zeros((n, n), np.float32), np.zeros((n, n), np.float32))
    s.set_block(T)
    if rows:
        s.set_tile_rows(rows)
    s.stimulate(disks)
    s.step(1500)
    u, v = s.read()
    s.close()
    op = {"xflip": lambda a: a[:, ::-1], "yflip": lambda a: a[::-1], "transpose": lambda a: a.T}[sym]
    assert v.max() > 0.05
    assert np.array_equal(u, op(u)) and np.array_equal(v, op(v))


def test_parameter_validation():
    s = rdc.Sim(16, 16, None, "fp32")
    good = dict(inputs.PARAMS_WORKLOAD)
    s.set_params(good)
    for key, bad in (("eps", 0.0), ("eps", -1.0), ("q", 0.0), ("D_u", -0.1), ("dt", 0.0),
                     ("dx", 0.0), ("f", float("nan")), ("dt", 0.1)):
        p = dict(good)
        p[key] = bad
        with pytest.raises(rdc.RdcError) as e:
            s.set_params(p)
        assert e.value.status == rdc.RDC_E_INVAL, (key, bad)
    p = dict(good)
    p["eps"] = float("inf")
    s.set_params(p)
    with pytest.raises(rdc.RdcError):
        s.set_block(13)
    s64 = rdc.Sim(16, 16, None, "fp64")
    with pytest.raises(rdc.RdcError):
        s64.set_block(9)
    s64.close()
    with pytest.raises(rdc.RdcError):
        s.step(-1)
    s.close()


# ------------------------------------------------------------------ circuit workload (small)

@pytest.fixture(scope="module")
def circuit_case():
    wl = inputs.circuit(n=512, seed=1002, steps=5000, ndisks=16, tile=128)
    run = oracle.Run(wl.u0, wl.v0, wl.phi, wl.params, track_arrival=True, track_unstable=True)
    run.run_schedule(wl.stimuli, wl.steps)
    return wl, run


@pytest.mark.parametrize("T,rows", [(1, 0), (8, 56)])
def test_circuit_fp64_bitwise(circuit_case, T, rows):
    wl, run = circuit_case
    print_case("circuit 512^2 fp64 T=%d rows=%d" % (T, rows))
    assert np.isfinite(run.u).all()
    s = make_sim(wl, "fp64", T=T, rows=rows, arrival=True)
    s.run_schedule(wl.stimuli, wl.steps)
    u, v = s.read()
    assert np.array_equal(u, run.u) and np.array_equal(v, run.v)
    assert np.array_equal(s.arrival(), run.arrival)
    s.close()


@pytest.mark.parametrize("T,rows", [(1, 0), (8, 80), (6, 64)])
def test_circuit_fp32_arrival_and_masked_field(circuit_case, T, rows):
    wl, run = circuit_case
    print_case("circuit 512^2 fp32 T=%d rows=%d" % (T, rows))
    s = make_sim(wl, "fp32", T=T, rows=rows, arrival=True)
    s.run_schedule(wl.stimuli, wl.steps)
    u, v = s.read()
    arr = s.arrival()
    s.close()
    nviol = arrival_violations(arr, run.arrival)
    print("  arrival violations %d, arrived %d" % (nviol, int((run.arrival < oracle.NEVER).sum())))
    assert arrival_within_one_cell(arr, run.arrival)
    mask = dilate(run.unstable.astype(bool), 1)
    du = masked_maxabs(u, run.u, mask)
    dv = masked_maxabs(v, run.v, mask)
    # Inhibitory background away from the channels: the period-2 orbit of
    # the phi = 0.2 cell map, where both precisions must sit in the same
    # phase.  What stays masked is the channels and their rim.
    p2 = background_far_from_channels(wl.phi)
    du2 = float(np.abs(u.astype(np.float64) - run.u)[p2].max())
    dv2 = float(np.abs(v.astype(np.float64) - run.v)[p2].max())
    rest = mask & ~p2
    print("  masked max|du|=%.3g max|dv|=%.3g, masked cells %.1f%%; period-2 background "
          "%.1f%% of cells, max|du|=%.3g max|dv|=%.3g; still masked %.1f%%"
          % (du, dv, 100.0 * mask.mean(), 100.0 * p2.mean(), du2, dv2, 100.0 * rest.mean()))
    assert du <= TOL and dv <= TOL
    assert du2 <= TOL and dv2 <= TOL
    assert p2.mean() > 0.7 and rest.mean() < 0.25
