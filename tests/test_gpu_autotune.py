"""The launch-shape autotuner: picks a measured candidate, caches it per
(arch, stepper sources, shape), leaves the caller's grid untouched, and the
tuned grid steps bit-identically to the one-step kernel."""
import json

import numpy as np
import pytest

from paper_1901_06535_amd import autotune, inputs, rdc

pytestmark = pytest.mark.gpu


def test_tune_sim_caches_and_keeps_state(tmp_path, monkeypatch):
    monkeypatch.setenv("RDC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    u, v, phi = inputs.random_state(600, 333, seed=5)
    s = rdc.Sim(600, 333, inputs.PARAMS_WORKLOAD, "fp32")
    s.set_phi(phi)
    s.write(u, v)
    s.step(3)
    before = s.read()
    rec = s.autotune(Ts=(4, 8), rows=(48, 56), launches=4)
    assert not rec["cached"] and (rec["T"], rec["rows"]) in {(4, 48), (4, 56), (8, 48), (8, 56)}
    assert set(rec["table"]) == {"T4_r48", "T4_r56", "T8_r48", "T8_r56"}
    assert rec["us_per_step"] == min(rec["table"].values())
    after = s.read()
    assert s.step_index == 3
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    data = json.load(open(tmp_path / "tune.json"))
    (key,) = data
    assert key.endswith("/single/600x333") and key.split("/")[0].startswith("gfx")
    again = s.autotune(Ts=(4, 8), rows=(48, 56), launches=4)
    assert again["cached"] and (again["T"], again["rows"]) == (rec["T"], rec["rows"])
    s.step(37)
    ref = rdc.Sim(600, 333, inputs.PARAMS_WORKLOAD, "fp32")
    ref.set_phi(phi)
    ref.write(u, v)
    ref.set_block(1)
    ref.step(40)
    a, b = s.read(), ref.read()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    s.close()
    ref.close()


def test_tune_batch(tmp_path, monkeypatch):
    monkeypatch.setenv("RDC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    specs = [(nx, ny, inputs.PARAMS_WORKLOAD) for nx, ny in ((64, 64), (300, 129), (257, 511))]
    b = rdc.BatchSim(specs)
    rec = b.autotune(Ts=(4, 8), rows=(48, 56), launches=4)
    assert (rec["T"], rec["rows"]) in {(4, 48), (4, 56), (8, 48), (8, 56)}
    assert b.autotune(Ts=(4, 8), rows=(48, 56), launches=4)["cached"]
    b.close()


def test_tune_fp64_sim_keys_by_precision_and_stays_bitwise(tmp_path, monkeypatch):
    """An FP64 grid is timed with FP64 kernels under its own cache key, and the
    tuned launch shape still gives the oracle's bits (the one-step FP64 run)."""
    monkeypatch.setenv("RDC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    u, v, phi = inputs.random_state(520, 300, seed=6, umax=0.02, vmax=0.02)
    s = rdc.Sim(520, 300, inputs.PARAMS_WORKLOAD, "fp64")
    s.set_phi(phi)
    s.write(u, v)
    rec = s.autotune(Ts=(4, 8), rows=(48, 64), launches=3)
    assert (rec["T"], rec["rows"]) in {(4, 48), (4, 64), (8, 48), (8, 64)}
    (key,) = json.load(open(tmp_path / "tune.json"))
    assert key.endswith("/single_fp64/520x300")
    s.stimulate([(260, 150, 6)])
    s.step(45)
    ref = rdc.Sim(520, 300, inputs.PARAMS_WORKLOAD, "fp64")
    ref.set_phi(phi)
    ref.write(u, v)
    ref.set_block(1)
    ref.stimulate([(260, 150, 6)])
    ref.step(45)
    a, b = s.read(), ref.read()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    s.close()
    ref.close()
