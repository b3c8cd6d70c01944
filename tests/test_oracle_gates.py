"""The paper's sanity circuits (Sec. 4), rebuilt from generated geometry and
run on the FP64 oracle: the qualitative outcomes the paper reports are the
pin.

  * Sec. 4.2: the chemical diode passes a wave from the flat (anode) side to
    the pointed (cathode) side and blocks the reverse direction.
  * Sec. 4.1: the coincidence-detector AND gate gives no output wave for a
    single input and an output wave when both inputs arrive together.
"""
import os

import pytest

import oracle
from paper_1901_06535_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fires(wl):
    r = oracle.run_workload(wl, track_arrival=True)
    x0, x1, y0, y1 = wl.extra["probe"]
    return bool((r.arrival[y0:y1, x0:x1] < oracle.NEVER).any())


def _window():
    vals = {}
    with open(os.path.join(GOLDEN, "and_gate_window.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals["lo"], vals["hi"]


@pytest.mark.parametrize("gap", [1, 2, 3])
def test_diode_passes_flat_to_tip(gap):
    assert _fires(inputs.diode_case("flat_to_tip", gap=gap))


@pytest.mark.parametrize("gap", [1, 2, 3])
def test_diode_blocks_tip_to_flat(gap):
    assert not _fires(inputs.diode_case("tip_to_flat", gap=gap))


def test_plain_channel_conducts_both_ways():
    """Control: without the cut the same channel carries the wave."""
    for d in ("flat_to_tip", "tip_to_flat"):
        assert _fires(inputs.diode_case(d, gap=0, tip=1, phi_gap=inputs.PHI_EXCITABLE))


def test_diode_gap_of_pure_inhibitor_blocks_both_ways():
    for d in ("flat_to_tip", "tip_to_flat"):
        assert not _fires(inputs.diode_case(d, gap=2, phi_gap=inputs.PHI_INHIBITORY))


@pytest.mark.parametrize("which", ["lo", "mid", "hi"])
def test_and_gate_truth_table_inside_window(which):
    lo, hi = _window()
    pg = {"lo": lo, "mid": round((lo + hi) / 2, 4), "hi": hi}[which]
    assert not _fires(inputs.and_case((1, 0), phi_gap=pg))
    assert not _fires(inputs.and_case((0, 1), phi_gap=pg))
    assert _fires(inputs.and_case((1, 1), phi_gap=pg))


def test_and_gate_default_gap_is_inside_window():
    lo, hi = _window()
    assert lo <= inputs.AND_PHI_GAP <= hi


def test_and_gate_outside_window():
    lo, hi = _window()
    assert _fires(inputs.and_case((1, 0), phi_gap=round(lo - 0.0005, 4)))   # gap too weak
    assert not _fires(inputs.and_case((1, 1), phi_gap=round(hi + 0.0005, 4)))  # too strong


@pytest.mark.parametrize("delay,expect", [(200, True), (400, True), (800, False)])
def test_and_gate_coincidence_tolerance(delay, expect):
    """Inputs that arrive a few hundred steps apart still collide above the
    output; far apart they pass each other's refractory tails and do not."""
    assert _fires(inputs.and_case((1, 1), delay=delay, steps=10000)) == expect
