"""The paper's sanity circuits (Sec. 4) on the GPU, against the FP64 oracle
on the same generated geometry: the FP64 kernel reproduces the oracle's
arrival map bit for bit, and the FP32 kernel at the benchmark's launch shape
gives the same gate outcome with arrival times within one cell.

  * Sec. 4.2 diode: flat (anode) side to pointed side passes, reverse blocked.
  * Sec. 4.1 AND gate: a single input gives no output wave, coincident
    inputs do.
"""
import numpy as np
import pytest

import oracle
from paper_1901_06535_amd import inputs, rdc

pytestmark = pytest.mark.gpu


def _gpu_arrival(wl, dtype, T=None, rows=56):
    s = rdc.Sim(wl.nx, wl.ny, wl.params, dtype)
    s.set_phi(wl.phi)
    s.write(wl.u0, wl.v0)
    if T:
        s.set_block(T)
        s.set_tile_rows(rows)
    s.enable_arrival(0.5)
    s.run_schedule(wl.stimuli, wl.steps)
    arr = s.arrival()
    s.read()                                  # raises on a non-finite state
    s.close()
    return arr


def _fires(arr, wl):
    x0, x1, y0, y1 = wl.extra["probe"]
    return bool((arr[y0:y1, x0:x1] < oracle.NEVER).any())


def _within_one_cell(a, b):
    """Every arrival of a lies within the 3x3 min..max of b, and vice versa."""
    ny, nx = a.shape
    def mm(x):
        p = np.pad(x.astype(np.int64), 1, mode="edge")
        win = np.stack([p[dy:dy + ny, dx:dx + nx] for dy in range(3) for dx in range(3)])
        return win.min(0), win.max(0)
    lo_b, hi_b = mm(b)
    lo_a, hi_a = mm(a)
    return bool(((a >= lo_b) & (a <= hi_b)).all() and ((b >= lo_a) & (b <= hi_a)).all())


CASES = [("diode_flat_to_tip", lambda: inputs.diode_case("flat_to_tip"), True),
         ("diode_tip_to_flat", lambda: inputs.diode_case("tip_to_flat"), False),
         ("and_10", lambda: inputs.and_case((1, 0)), False),
         ("and_01", lambda: inputs.and_case((0, 1)), False),
         ("and_11", lambda: inputs.and_case((1, 1)), True)]


@pytest.mark.parametrize("name,make,expect", CASES, ids=[c[0] for c in CASES])
def test_gate_on_gpu_matches_oracle(name, make, expect):
    wl = make()
    ref = oracle.run_workload(wl, track_arrival=True).arrival
    assert _fires(ref, wl) == expect                   # the oracle's own pin
    a64 = _gpu_arrival(wl, "fp64")
    assert np.array_equal(a64, ref)
    for T, rows in ((8, 56), (10, 64), (11, 64)):
        a32 = _gpu_arrival(wl, "fp32", T=T, rows=rows)
        assert _fires(a32, wl) == expect, (T, rows)
        assert _within_one_cell(a32, ref), (T, rows)
