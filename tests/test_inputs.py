"""Seeded input generators: determinism, shapes, and the recipe's invariants."""
import numpy as np

from paper_1901_06535_amd import inputs


def test_single_disk_is_deterministic_and_in_range():
    a, b = inputs.single_disk(), inputs.single_disk()
    assert a.manifest_json() == b.manifest_json()
    s = a.stimuli[0]
    assert 6 <= s.cx <= 249 and 6 <= s.cy <= 249 and s.r == 5 and s.step == 0
    assert a.phi.dtype == np.float32 and np.all(a.phi == np.float32(0.054))
    assert inputs.single_disk(seed=7).manifest_json() != a.manifest_json()


def test_uniform_random_phi_range_and_disks():
    wl = inputs.uniform_random_phi(n=512, seed=1003)
    assert wl.phi.min() >= np.float32(0.04) and wl.phi.max() < np.float32(0.08)
    assert len(wl.stimuli) == 64 and all(s.step == 0 for s in wl.stimuli)
    assert wl.manifest_json() == inputs.uniform_random_phi(n=512, seed=1003).manifest_json()


def test_circuit_map_values_and_stimuli():
    wl = inputs.circuit(n=1024, seed=1002, steps=10000, ndisks=64)
    vals = set(np.unique(wl.phi).tolist())
    allowed = {np.float32(v).item() for v in
               (inputs.PHI_INHIBITORY, inputs.PHI_EXCITABLE, inputs.DIODE_PHI_GAP,
                inputs.AND_PHI_GAP)}
    assert vals <= allowed
    assert np.float32(inputs.PHI_EXCITABLE).item() in vals
    steps = [s.step for s in wl.stimuli]
    assert steps == sorted(steps) and 0 <= steps[0] and steps[-1] < 10000
    for s in wl.stimuli:
        assert wl.phi[s.cy, s.cx] == np.float32(inputs.PHI_EXCITABLE)
    assert wl.manifest_json() == inputs.circuit(n=1024, seed=1002, steps=10000,
                                                ndisks=64).manifest_json()


def test_circuit_disk_schedule_spans_the_run_and_keeps_spacing():
    """Input disks land at steps spread over the whole run (not only at its
    start) and every pair, earlier or later, keeps the space-time spacing."""
    wl = inputs.circuit(n=4096, seed=1002, steps=10000, ndisks=256)
    t = np.array([s.step for s in wl.stimuli])
    assert len(t) == 256 and list(t) == sorted(t)
    # quartiles of a uniform sample of 256 from [0, 10,000) lie within +-800
    # of 2,500 / 5,000 / 7,500 with overwhelming probability
    q = np.percentile(t, [25, 50, 75])
    assert np.all(np.abs(q - np.array([2500, 5000, 7500])) < 800), q
    assert t[-1] > 9000
    for i, a in enumerate(wl.stimuli):
        for b in wl.stimuli[i + 1:]:
            assert inputs.spacing_ok(a.step, a.cx, a.cy, b.step, b.cx, b.cy)


def test_circuit_channels_join_across_tiles():
    """Every motif puts its channel on the tile centre lines, so a channel that
    reaches a tile edge does so at the centre band of that edge."""
    wl = inputs.circuit(n=1024, seed=5, ndisks=8)
    act = wl.phi != np.float32(inputs.PHI_INHIBITORY)
    for t in range(1, 4):
        edge = act[:, t * 256 - 1]
        band = np.zeros(1024, dtype=bool)
        for k in range(4):
            band[k * 256 + 120:k * 256 + 136] = True
        assert not (edge & ~band).any()


def test_batch_sweep_sizes_and_params():
    sims, steps = inputs.batch_sweep(count=64, seed=1004)
    assert steps == 5000 and len(sims) == 64
    for s in sims:
        assert 64 <= s.nx <= 1024 and 64 <= s.ny <= 1024
        assert 0.02 <= s.params["eps"] <= 0.03
        assert 1 <= len(s.stimuli) <= 4
        assert s.phi.shape == (s.ny, s.nx)
    again, _ = inputs.batch_sweep(count=64, seed=1004)
    assert all(a.nx == b.nx and np.array_equal(a.phi, b.phi) for a, b in zip(sims, again))


def test_pitch_is_multiple_of_64():
    for nx in (1, 63, 64, 65, 4096, 16383):
        p = inputs.pitch_for(nx)
        assert p % 64 == 0 and p >= nx and p - nx < 64
