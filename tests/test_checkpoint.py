"""Checkpoint files (CPU): arrays and manifest round-trip, and any change to
an array, the array set or the format is refused on load."""
import json

import numpy as np
import pytest

from paper_1901_06535_amd import checkpoint


def _arrays():
    rng = np.random.default_rng(1)
    return {"u": rng.random((5, 7)).astype(np.float32), "v": rng.random((5, 7)),
            "arrival": rng.integers(0, 100, (5, 7)).astype(np.int32)}


def test_round_trip(tmp_path):
    p = str(tmp_path / "ck")
    a = _arrays()
    checkpoint.write(p, a, {"nx": 7, "ny": 5, "step": 130, "params": {"eps": 0.022}})
    b, meta = checkpoint.read(p)
    assert sorted(b) == sorted(a)
    for k in a:
        assert b[k].dtype == a[k].dtype and np.array_equal(b[k], a[k])
    assert meta["step"] == 130 and meta["params"] == {"eps": 0.022} and meta["format"] == 1


def test_a_changed_array_is_refused(tmp_path):
    p = str(tmp_path / "ck")
    a = _arrays()
    checkpoint.write(p, a, {"step": 1})
    a["u"][2, 3] += 1e-6
    np.savez(p + ".npz", **a)
    with pytest.raises(ValueError, match="digest"):
        checkpoint.read(p)


def test_a_missing_array_or_other_format_is_refused(tmp_path):
    p = str(tmp_path / "ck")
    a = _arrays()
    checkpoint.write(p, a, {"step": 1})
    del a["arrival"]
    np.savez(p + ".npz", **a)
    with pytest.raises(ValueError, match="manifest lists"):
        checkpoint.read(p)
    checkpoint.write(p, _arrays(), {"step": 1})
    man = json.load(open(p + ".json"))
    man["format"] = 99
    json.dump(man, open(p + ".json", "w"))
    with pytest.raises(ValueError, match="format"):
        checkpoint.read(p)
