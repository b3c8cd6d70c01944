"""Checkpoint and resume of a stepper context: the snapshot of Sec. 3.1 made
resumable.  The state planes (u, v), phi and the optional arrival-time and
timelapse planes go into one .npz; a JSON manifest beside it records the
grid, precision, Eq. (1) parameters, step index, an optional seed and the
sha256 of every array, and is checked on load (a changed or missing array is
an error).  Only numbers are stored: loading executes nothing from the files.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Tuple

import numpy as np

FORMAT = 1


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def write(path: str, arrays: Dict[str, np.ndarray], meta: Dict) -> None:
    """Write `path`.npz (the arrays) and `path`.json (meta + digests)."""
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp + ".npz", "wb") as fh:
        np.savez(fh, **arrays)
    man = dict(meta, format=FORMAT, arrays=sorted(arrays),
               sha256={k: _sha(v) for k, v in arrays.items()},
               dtypes={k: str(v.dtype) for k, v in arrays.items()})
    with open(tmp + ".json", "w") as fh:
        json.dump(man, fh, indent=1, sort_keys=True)
    os.replace(tmp + ".npz", path + ".npz")
    os.replace(tmp + ".json", path + ".json")


def read(path: str) -> Tuple[Dict[str, np.ndarray], Dict]:
    """The arrays and manifest written by `write`, after checking them."""
    with open(path + ".json") as fh:
        meta = json.load(fh)
    if meta.get("format") != FORMAT:
        raise ValueError("%s.json: not a checkpoint of format %d" % (path, FORMAT))
    with np.load(path + ".npz", allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    if sorted(arrays) != meta["arrays"]:
        raise ValueError("%s.npz holds %s, the manifest lists %s"
                         % (path, sorted(arrays), meta["arrays"]))
    for k, v in arrays.items():
        if str(v.dtype) != meta["dtypes"][k] or _sha(v) != meta["sha256"][k]:
            raise ValueError("%s.npz: array %r does not match its manifest digest" % (path, k))
    return arrays, meta
