"""Checkpoint / resume on the GPU: a run saved at some step and resumed in a
fresh context (state, phi, step index, arrival map, timelapse) ends bit for
bit where the uninterrupted run ends, in both precisions."""
import numpy as np
import pytest

from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,T", [("fp32", 8), ("fp64", 8), ("fp32", 1)])
def test_resume_from_checkpoint_is_bitwise(tmp_path, dtype, T):
    nx, ny, steps, cut = 300, 220, 300, 133
    print("[case] checkpoint %s T=%d" % (dtype, T), flush=True)
    u, v, phi = inputs.random_state(nx, ny, seed=41, umax=0.02, vmax=0.02, phi_lo=0.04,
                                    phi_hi=0.08)
    sched = [(0, 40, 50, 6), (90, 250, 160, 5), (150, 120, 20, 4), (260, 10, 210, 3)]

    def start():
        s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, dtype)
        s.set_phi(phi)
        s.write(u, v)
        s.set_block(T)
        s.enable_arrival(0.5)
        s.enable_timelapse(7)
        return s

    ref = start()
    ref.run_schedule(sched, steps)
    want = list(ref.read()) + [ref.arrival(), ref.timelapse()]
    ref.close()

    a = start()
    a.run_schedule(sched, cut)
    a.save_checkpoint(str(tmp_path / "ck"), seed=41)
    a.close()
    b = rdc.Sim.from_checkpoint(str(tmp_path / "ck"))
    assert b.step_index == cut and b.dtype == dtype
    b.set_block(T)
    b.run_schedule(sched, steps)
    got = list(b.read()) + [b.arrival(), b.timelapse()]
    assert b.step_index == steps
    b.close()
    for x, y in zip(got, want):
        assert np.array_equal(x, y)
    assert (want[2] < np.iinfo(np.int32).max).sum() > 100     # fronts arrived after the cut
