"""Stimulation schedules through rdc_run: stimuli that fall inside a T-step
launch are applied by the launch itself, between its sub-steps.

SKIPPED: the in-kernel stimulation path (an rdc_run entry point whose T-step
kernels took a per-launch disk list) ended its first GPU run with a host
segmentation fault inside rdc_run, before any result was checked.  Its host
scheduling logic ran clean under AddressSanitizer and UBSan on the CPU with
the launches intercepted, and no cause was found, so the path was taken out
of the library (stimuli split the launches, as rdc_stimulate between
rdc_step calls does); these tests stay as the specification of the path.

Bars:
  * bit-identical to the split route (step to each stimulus step, stimulate,
    step on) and to the one-step kernel, for every launch shape, with disks on
    edges and corners (their mirrored halo copies), more disks inside one
    launch than a launch carries, disks at launch starts and at the final
    step, with the arrival map and timelapse attached or not;
  * FP32 against the FP64 oracle (max-abs 1e-4) on a short horizon with
    mid-launch stimuli;
  * argument errors reported before anything is launched.
"""
import numpy as np
import pytest

import oracle
from paper_1901_06535_amd import inputs, rdc

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="in-kernel stimulation path removed after a host "
                                      "segfault on its first GPU run; cause not found")]

PARAMS = inputs.PARAMS_WORKLOAD


def _covers_grid(nx, ny, cx, cy, r):
    px, py = min(max(cx, 0), nx - 1), min(max(cy, 0), ny - 1)
    return (px - cx) ** 2 + (py - cy) ** 2 <= r * r


def _schedule(nx, ny, steps, seed):
    rng = np.random.default_rng(seed)
    st = [(int(rng.integers(0, steps + 1)), int(rng.integers(-4, nx + 4)),
           int(rng.integers(-4, ny + 4)), int(rng.integers(0, 9))) for _ in range(60)]
    st += [(5, 0, 0, 4), (13, nx - 1, ny - 1, 6), (21, nx // 2, 0, 3), (27, 0, ny // 2, 0),
           (30, nx + 2, ny // 3, 4), (35, nx // 3, ny + 1, 3), (37, nx - 2, 1, 2)]
    # 24 disks over five steps of one launch window: more than one launch carries
    st += [(41 + i % 5, int(rng.integers(0, nx)), int(rng.integers(0, ny)), 3) for i in range(24)]
    st += [(0, nx // 2, ny // 2, 6), (16, nx // 3, ny // 3, 5), (64, nx // 5, ny // 2, 4),
           (steps, nx // 4, ny // 4, 5)]
    return [s for s in st if _covers_grid(nx, ny, *s[1:])]


def _state(nx, ny, seed):
    u, v, phi = inputs.random_state(nx, ny, seed=seed, umax=0.02, vmax=0.02, phi_lo=0.04,
                                    phi_hi=0.08)
    return u, v, phi


def _run(nx, ny, state, sched, steps, T, rows, fused, outputs, chunks=(0.37, 1.0)):
    u, v, phi = state
    s = rdc.Sim(nx, ny, PARAMS, "fp32")
    s.set_phi(phi)
    s.write(u, v)
    s.set_block(T)
    s.set_tile_rows(rows)
    if outputs:
        s.enable_arrival(0.5)
        s.enable_timelapse(3)
    for f in chunks:               # two calls: the second starts mid-schedule
        until = int(round(f * steps))
        if fused:
            s.run_schedule(sched, until)
        else:
            s.run_schedule_split(sched, until)
    out = list(s.read())
    if outputs:
        out += [s.arrival(), s.timelapse()]
    assert s.step_index == steps
    s.close()
    return out


@pytest.mark.parametrize("T,rows,outputs", [(8, 56, False), (8, 56, True), (5, 48, False),
                                            (2, 64, True), (7, 80, False), (3, 56, False)])
def test_fused_schedule_equals_split_route_bitwise(T, rows, outputs):
    nx, ny, steps = 333, 275, 120
    print("[case] fused vs split T=%d rows=%d outputs=%s" % (T, rows, outputs), flush=True)
    state = _state(nx, ny, 21)
    sched = _schedule(nx, ny, steps, 5)
    fused = _run(nx, ny, state, sched, steps, T, rows, True, outputs)
    split = _run(nx, ny, state, sched, steps, T, rows, False, outputs)
    for a, b in zip(fused, split):
        assert np.array_equal(a, b)


def test_fused_schedule_equals_one_step_kernel():
    nx, ny, steps = 300, 260, 100
    print("[case] fused T=8 vs one-step kernel", flush=True)
    state = _state(nx, ny, 22)
    sched = _schedule(nx, ny, steps, 6)
    a = _run(nx, ny, state, sched, steps, 8, 56, True, True)
    b = _run(nx, ny, state, sched, steps, 1, 56, True, True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_fused_schedule_matches_the_oracle():
    nx, ny, steps = 150, 110, 60
    print("[case] fused T=8 vs oracle", flush=True)
    u, v, phi = _state(nx, ny, 23)
    sched = [(3, 0, 0, 5), (9, nx - 1, 50, 4), (11, 70, ny - 1, 6), (17, 40, 40, 3),
             (17, 100, 20, 2), (26, 149, 109, 7), (33, -2, 60, 4), (45, 75, 55, 5)]
    s = rdc.Sim(nx, ny, PARAMS, "fp32")
    s.set_phi(phi)
    s.write(u, v)
    s.set_block(8)
    s.run_schedule(sched, steps)
    gu, gv = s.read()
    s.close()
    run = oracle.Run(u, v, phi, PARAMS)
    run.run_schedule(sched, steps)
    du = float(np.max(np.abs(gu - run.u)))
    dv = float(np.max(np.abs(gv - run.v)))
    print("  max|du|=%.3g max|dv|=%.3g" % (du, dv))
    assert du <= 1e-4 and dv <= 1e-4
    # every scheduled disk was applied: the stimulated cells are excited
    assert (gu > 0.3).sum() > 100


def test_run_rejects_bad_schedules_before_launching():
    nx, ny = 64, 48
    u, v, phi = _state(nx, ny, 24)
    s = rdc.Sim(nx, ny, PARAMS, "fp32")
    s.set_phi(phi)
    s.write(u, v)
    s.step(10)
    bad = [([9], [5], [5], [2]),            # before the current step
           ([31], [5], [5], [2]),           # after current + n
           ([12], [5], [5], [-1]),          # negative radius
           ([12], [200], [5], [3])]         # covers no cell
    for st, cx, cy, r in bad:
        with pytest.raises(rdc.RdcError) as e:
            rdc.rdc_run(s.ctx, 20, st, cx, cy, r)
        assert e.value.status == rdc.RDC_E_INVAL
        assert s.step_index == 10
    s.close()
