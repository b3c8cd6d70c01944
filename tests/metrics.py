"""Comparison metrics for stepper parity (test infrastructure).

The scheme is Euler-unstable in refractory tails and on strongly inhibitory
substrate, where rounding differences grow chaotically; the oracle flags
those cells (Euler factor below -1).  Parity is therefore stated as
  * full-field max-abs up to the first such step,
  * max-abs outside a dilation of the flagged cells at the horizon,
  * arrival times (first step with u >= theta) equal to within one cell,
  * FP64 kernels bit-identical to the oracle at every horizon.
"""
import numpy as np

NEVER = np.iinfo(np.int32).max


def dilate(mask: np.ndarray, k: int = 1) -> np.ndarray:
    """Chebyshev dilation of a boolean mask by k cells."""
    out = mask.astype(bool).copy()
    for _ in range(k):
        m = out.copy()
        m[1:, :] |= out[:-1, :]
        m[:-1, :] |= out[1:, :]
        m2 = m.copy()
        m2[:, 1:] |= m[:, :-1]
        m2[:, :-1] |= m[:, 1:]
        out = m2
    return out


def _neigh_minmax(a: np.ndarray):
    """Min and max of a over each cell's 3x3 (Moore) neighbourhood."""
    p = np.pad(a.astype(np.int64), 1, mode="edge")
    ny, nx = a.shape
    stack = np.stack([p[j:j + ny, i:i + nx] for j in range(3) for i in range(3)])
    return stack.min(0), stack.max(0)


def arrival_within_one_cell(test: np.ndarray, ref: np.ndarray) -> bool:
    """Each arrival time of ``test`` lies between the min and max of ``ref``
    over the cell's 3x3 neighbourhood, and the other way round."""
    lo, hi = _neigh_minmax(ref)
    t = test.astype(np.int64)
    ok1 = np.all((t >= lo) & (t <= hi))
    lo2, hi2 = _neigh_minmax(test)
    r = ref.astype(np.int64)
    ok2 = np.all((r >= lo2) & (r <= hi2))
    return bool(ok1 and ok2)


def arrival_violations(test: np.ndarray, ref: np.ndarray) -> int:
    lo, hi = _neigh_minmax(ref)
    t = test.astype(np.int64)
    return int(np.count_nonzero((t < lo) | (t > hi)))


def masked_maxabs(a: np.ndarray, b: np.ndarray, mask_out: np.ndarray = None) -> float:
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    if mask_out is not None:
        d = d[~mask_out]
    return float(d.max()) if d.size else 0.0


def front_error(a: np.ndarray, b: np.ndarray, theta: float = 0.5, kmax: int = 64) -> int:
    """Smallest k with {a >= theta} inside the k-dilation of {b >= theta} and
    vice versa (Chebyshev); kmax+1 if larger."""
    fa, fb = a >= theta, b >= theta
    da, db = fa.copy(), fb.copy()
    for k in range(kmax + 1):
        if not (fa & ~db).any() and not (fb & ~da).any():
            return k
        da, db = dilate(da, 1), dilate(db, 1)
    return kmax + 1


def background_far_from_channels(phi: np.ndarray, d: int = 4, phi_bg: float = 0.2) -> np.ndarray:
    """Cells of the phi = phi_bg background at Chebyshev distance >= d from
    any other cell.  On the phi = 0.2 background the homogeneous state is on
    a period-2 orbit of the cell map; waves in the channels perturb cells
    this far away by less than 1e-4 (the FP64 oracle's state there is within
    4e-5 of the homogeneous orbit at d = 4 on the 512^2 circuit)."""
    from scipy.ndimage import distance_transform_cdt
    bg = phi == np.float32(phi_bg)
    return bg & (distance_transform_cdt(bg, metric="chessboard") >= d)
