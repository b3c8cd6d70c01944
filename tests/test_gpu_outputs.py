"""Outputs fused into the stepping kernels: the timelapse max-projection
(and its coexistence with the arrival map), against the FP64 oracle and
across launch shapes."""
import numpy as np
import pytest

import oracle
from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu


def _state(nx, ny, seed):
    u, v, phi = inputs.random_state(nx, ny, seed=seed)
    return u, v, phi


@pytest.mark.parametrize("rate,T", [(1, 1), (3, 1), (7, 1), (1, 8), (3, 5), (7, 8)])
def test_fp64_timelapse_bitwise_equals_oracle(rate, T):
    nx, ny = 96, 80
    u, v, phi = _state(nx, ny, 31)
    s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, "fp64")
    s.set_block(T)
    s.set_phi(phi)
    s.write(u, v)
    s.stimulate([(40, 30, 5)])
    s.step(4)
    s.enable_timelapse(rate)
    s.enable_arrival(0.5)
    s.step(61)
    s.stimulate([(70, 60, 4)])
    s.step(140)
    got = s.timelapse()
    arr = s.arrival()
    s.close()
    run = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD)
    run.stimulate([(40, 30, 5)])
    run.advance(4)
    run.track_timelapse(rate)
    run.advance(61)
    run.stimulate([(70, 60, 4)])
    run.advance(140)
    assert np.array_equal(got, run.timelapse)
    ref_arr = oracle.Run(u, v, phi, inputs.PARAMS_WORKLOAD, track_arrival=True)
    ref_arr.stimulate([(40, 30, 5)])
    ref_arr.advance(4)
    assert (run.timelapse >= 0.5).any()
    # the arrival map attached at step 4 still matches (both outputs in one kernel)
    r2 = oracle.Run(ref_arr.u, ref_arr.v, phi, inputs.PARAMS_WORKLOAD, track_arrival=True)
    r2.step_index = 4
    r2.arrival[:] = np.where(ref_arr.u >= 0.5, 4, oracle.NEVER)
    r2.advance(61)
    r2.stimulate([(70, 60, 4)])
    r2.advance(140)
    assert np.array_equal(arr, r2.arrival)


@pytest.mark.parametrize("T,rows", [(3, 48), (8, 56), (8, 80), (5, 64),
                                    (11, rdc.RDC_TILE_STREAM)])
@pytest.mark.parametrize("rate", [1, 4, 5])
def test_fp32_timelapse_is_launch_shape_invariant(T, rows, rate):
    """Every (T, tile height) gives the one-step kernel's timelapse bit for
    bit, also when the rate does not divide T and around the stimulus split
    (with the row pipelines chosen, the steps before the timelapse is
    attached run on them, and the launches while it records on the LDS
    tiles)."""
    nx, ny = 333, 275
    u, v, phi = _state(nx, ny, 37)
    out = []
    for blk, r in ((1, 56), (T, rows)):
        s = rdc.Sim(nx, ny, inputs.PARAMS_WORKLOAD, "fp32")
        s.set_phi(phi)
        s.write(u, v)
        s.set_block(blk)
        s.set_tile_rows(r)
        s.stimulate([(100, 100, 6)])
        s.step(3)
        s.enable_timelapse(rate)
        s.step(47)
        s.stimulate([(250, 200, 5)])
        s.step(53)
        out.append((s.timelapse(), s.read()[0]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    if 103 % rate == 0:                       # the final state is a frame
        assert (out[0][0] >= out[0][1]).all()


def test_timelapse_detach_and_validation():
    import torch
    s = rdc.Sim(64, 64, inputs.PARAMS_WORKLOAD, "fp32")
    with pytest.raises(rdc.RdcError):
        rdc.rdc_set_timelapse(s.ctx, s.planes[0].data_ptr(), s.pitch, 0)
    with pytest.raises(rdc.RdcError):
        rdc.rdc_set_timelapse(s.ctx, s.planes[0].data_ptr() + 4, s.pitch, 1)
    s.enable_timelapse(2)
    s.step(4)
    before = s.timelapse().copy()
    rdc.rdc_set_timelapse(s.ctx, None, 0, 1)
    s.stimulate([(30, 30, 5)])
    s.step(6)
    torch.cuda.synchronize()
    assert np.array_equal(s.timelapse(), before)      # detached: no longer written
    s.close()
