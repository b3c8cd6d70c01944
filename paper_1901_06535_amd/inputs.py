"""Seeded synthetic inputs for the Oregonator stepper.

This module draws geometry and random numbers only.  It holds no step of the
method's arithmetic (no reaction term, no Laplacian, no stimulation rule), so
both the FP64 oracle and the HIP path may take their inputs from it.

What the inputs stand for:
  * the model and its default parameters: Sec. 2, Eq. (1) and Table 1;
  * the drawn excitability map phi (active vs. passive substrate) and the
    line-width / background presets: Sec. 3;
  * the circuits the paper rebuilds (coincidence-detector AND gate, Agladze
    diode): Sec. 4.1 and 4.2.  Their drawings are not available, so the
    geometry here is generated and parameterised (see ``diode_case`` and
    ``and_case``).
  * "catalytic stimulation" (Sec. 2) is described by disks
    ``(step, cx, cy, r)``; the rule that applies a disk lives with the
    implementations, not here.

Every array is float32 (so the FP32 kernel, the FP64 kernel and the FP64
oracle start from identical values: the oracle widens them exactly) and every
draw goes through ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Table 1 of the paper (Sec. 2): default parameter values.
PARAMS_TABLE1 = dict(eps=0.0243, f=1.4, q=0.002, D_u=0.45, dt=0.001, dx=0.25)
PHI_ACTIVE_TABLE1 = 0.054
PHI_PASSIVE_TABLE1 = 0.0975

# The measured workloads use eps=0.022, D_u=1.0 and an inhibitory
# background phi=0.2, with the remaining Table 1 values.
PARAMS_WORKLOAD = dict(eps=0.022, f=1.4, q=0.002, D_u=1.0, dt=0.001, dx=0.25)
PHI_EXCITABLE = 0.054
PHI_INHIBITORY = 0.2
CHANNEL_WIDTH = 16
STIM_RADIUS = 5
# Upper bound on the wave-front speed in cells per step at the workload
# parameters (fronts move about 0.022 cells/step), and the extra distance
# kept between input disks.  Used only to space input disks in space-time.
FRONT_SPEED_BOUND = 0.03
DISK_MARGIN = 40

# Agladze-style diode and coincidence AND gate (Sec. 4), geometry constants.
DIODE_PHI_GAP = 0.0975
DIODE_GAP = 2
DIODE_TIP = 8
# Passive gap between the AND gate's input and output channels; the default is
# the middle of the window in which the gate fires on 11 but not on 10 / 01.
# ``tests/golden/and_gate_window.txt`` holds the calibrated window.
AND_GAP_ROWS = 2
AND_PHI_GAP = 0.125


@dataclasses.dataclass
class Stimulus:
    """A disk of catalytic stimulation applied before step ``step``."""
    step: int
    cx: int  # column (x)
    cy: int  # row (y)
    r: int


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    params: Dict[str, float]
    phi: np.ndarray          # (ny, nx) float32
    u0: np.ndarray           # (ny, nx) float32
    v0: np.ndarray           # (ny, nx) float32
    stimuli: List[Stimulus]
    steps: int
    seed: int
    extra: Dict[str, object] = dataclasses.field(default_factory=dict)

    def manifest(self) -> Dict[str, object]:
        """JSON-able record of everything that defines the run."""
        def sha(a: np.ndarray) -> str:
            return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
        return {
            "name": self.name, "nx": self.nx, "ny": self.ny,
            "params": dict(self.params), "seed": self.seed, "steps": self.steps,
            "phi_sha256": sha(self.phi), "u0_sha256": sha(self.u0),
            "v0_sha256": sha(self.v0),
            "stimuli": [dataclasses.astuple(s) for s in self.stimuli],
            "extra": {k: v for k, v in self.extra.items()
                      if isinstance(v, (int, float, str, bool, list))},
        }

    def manifest_json(self) -> str:
        return json.dumps(self.manifest(), sort_keys=True)

    def stimuli_by_step(self) -> List[Tuple[int, List[Stimulus]]]:
        """Stimuli grouped by the step before which they are applied."""
        out: Dict[int, List[Stimulus]] = {}
        for s in self.stimuli:
            out.setdefault(int(s.step), []).append(s)
        return sorted(out.items())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _disk_fits(active: np.ndarray, r: int) -> np.ndarray:
    """Cells whose whole radius-r disk ((x-cx)^2 + (y-cy)^2 <= r^2) lies on
    ``active`` cells inside the grid: where an input disk can be placed
    without catalysing the inhibitory background."""
    from scipy.ndimage import binary_erosion
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    foot = (xx * xx + yy * yy) <= r * r
    return binary_erosion(active, structure=foot, border_value=0)


def _zeros(ny: int, nx: int) -> np.ndarray:
    return np.zeros((ny, nx), dtype=np.float32)


# --------------------------------------------------------------------------
# Workloads of the measured configurations
# --------------------------------------------------------------------------

def single_disk(n: int = 256, seed: int = 1001, steps: int = 1000) -> Workload:
    """256x256 grid, phi = 0.054 everywhere, u = v = 0 except one r=5 disk at a
    seeded position (its centre drawn from U{6..n-7}^2); 1,000 steps."""
    rng = _rng(seed)
    cx, cy = (int(c) for c in rng.integers(6, n - 6, size=2))
    phi = np.full((n, n), PHI_EXCITABLE, dtype=np.float32)
    return Workload("single_disk_%d" % n, n, n, dict(PARAMS_WORKLOAD), phi,
                    _zeros(n, n), _zeros(n, n), [Stimulus(0, cx, cy, STIM_RADIUS)],
                    steps, seed)


def uniform_random_phi(n: int = 16384, seed: int = 1003, steps: int = 2000,
                       ndisks: int = 64, ny: Optional[int] = None) -> Workload:
    """phi ~ U[0.04, 0.08) i.i.d. per cell, ``ndisks`` r=5 disks at uniformly
    random centres at t=0, u = v = 0 elsewhere (the 16384^2 scale case)."""
    ny = n if ny is None else ny
    rng = _rng(seed)
    phi = rng.random((ny, n), dtype=np.float32)
    phi *= np.float32(0.04)
    phi += np.float32(0.04)
    cx = rng.integers(0, n, size=ndisks)
    cy = rng.integers(0, ny, size=ndisks)
    stim = [Stimulus(0, int(x), int(y), STIM_RADIUS) for x, y in zip(cx, cy)]
    return Workload("uniform_phi_%dx%d" % (n, ny), n, ny, dict(PARAMS_WORKLOAD), phi,
                    _zeros(ny, n), _zeros(ny, n), stim, steps, seed)


# Label values of the circuit map.
_BG, _CH, _DIODE_GAP, _AND_GAP = 0, 1, 2, 3
_MOTIFS = ("h", "v", "cross", "corner", "diode", "and")


def _draw_motif(lab: np.ndarray, motif: str, rot: int, rng: np.random.Generator,
                tile: int) -> None:
    """Draw one motif into a (tile x tile) label block (in place), then rotate."""
    w = CHANNEL_WIDTH
    c0 = tile // 2 - w // 2          # channel band [c0, c0 + w)
    c1 = c0 + w
    blk = np.zeros((tile, tile), dtype=np.uint8)
    if motif == "h":
        blk[c0:c1, :] = _CH
    elif motif == "v":
        blk[:, c0:c1] = _CH
    elif motif == "cross":
        blk[c0:c1, :] = _CH
        blk[:, c0:c1] = _CH
    elif motif == "corner":
        blk[c0:c1, :c1] = _CH
        blk[c0:, c0:c1] = _CH
    elif motif == "diode":
        blk[c0:c1, :] = _CH
        xl = tile // 2 - (DIODE_GAP + DIODE_TIP) // 2
        _draw_diode_gap(blk, c0, xl, DIODE_GAP, DIODE_TIP)
    elif motif == "and":
        blk[c0:c1, :] = _CH
        blk[c1:c1 + AND_GAP_ROWS, c0:c1] = _AND_GAP
        blk[c1 + AND_GAP_ROWS:, c0:c1] = _CH
    else:  # pragma: no cover - guarded by _MOTIFS
        raise ValueError(motif)
    lab[:, :] = np.rot90(blk, rot)


def _draw_diode_gap(blk: np.ndarray, row0: int, xl: int, gap: int, tip: int,
                    width: int = CHANNEL_WIDTH) -> None:
    """Cut an Agladze-style diode into a horizontal channel occupying rows
    [row0, row0+width): the channel ends flat at column ``xl``; ``gap``
    passive columns (label ``_DIODE_GAP``) follow across the channel's full
    width; then an active tip whose half-width grows linearly from the gap to
    the full channel over ``tip`` columns.  Channel cells beside the tip that
    it does not cover become background."""
    blk[row0:row0 + width, xl:xl + gap + tip] = _BG
    blk[row0:row0 + width, xl:xl + gap] = _DIODE_GAP
    ic = row0 + (width - 1) / 2.0
    for k in range(tip):
        half = (k + 0.5) * (width / 2.0) / tip
        for i in range(row0, row0 + width):
            if abs(i - ic) <= half:
                blk[i, xl + gap + k] = _CH


def spacing_ok(t: int, x: int, y: int, tj: int, xj: int, yj: int) -> bool:
    """Whether two input disks (step t, centre (x, y)) and (tj, (xj, yj))
    keep the space-time spacing: the later one lands where no wave of the
    earlier one can be yet, |x - x_j| >= FRONT_SPEED_BOUND * |t - t_j| +
    DISK_MARGIN (Euclidean distance bounds the path along the channels from
    below)."""
    return bool(np.hypot(x - xj, y - yj) >= FRONT_SPEED_BOUND * abs(t - tj) + DISK_MARGIN)


def _spaced_disks(rng: np.random.Generator, active: np.ndarray, steps: int,
                  ndisks: int, order: str = "drawn") -> List[Stimulus]:
    """Up to ``ndisks`` r=5 input disks wholly inside the ``active`` cells at
    steps drawn uniformly from [0, steps): 8 * ndisks candidates (step,
    centre) are drawn independently and taken in the order drawn
    (``order="drawn"``, which spreads the kept disks over the whole run) or
    in time order (``order="time"``, which fills the budget with the
    earliest ones), each kept if it keeps the space-time spacing
    (``spacing_ok``) with every disk kept so far, earlier or later in time;
    the kept disks are returned in time order.  (Catalysing medium that an
    earlier wave has left refractory drives forward Euler at dt = 0.001 into
    divergence.)"""
    fits = _disk_fits(active, STIM_RADIUS)
    fy, fx = np.nonzero(fits)
    cand_t = rng.integers(0, steps, size=8 * ndisks)
    cand_p = rng.integers(0, fy.size, size=8 * ndisks)
    if order == "time":
        pick = np.argsort(cand_t, kind="stable")
    elif order == "drawn":
        pick = np.arange(cand_t.size)
    else:
        raise ValueError(order)
    kept = []
    for c in pick:
        t, y, x = int(cand_t[c]), int(fy[cand_p[c]]), int(fx[cand_p[c]])
        if all(spacing_ok(t, x, y, tj, xj, yj) for (tj, yj, xj) in kept):
            kept.append((t, y, x))
            if len(kept) == ndisks:
                break
    kept.sort()
    return [Stimulus(t, x, y, STIM_RADIUS) for t, y, x in kept]


def circuit(n: int = 4096, seed: int = 1002, steps: int = 10000, ndisks: int = 256,
            tile: int = 256, and_phi_gap: float = AND_PHI_GAP,
            disk_order: str = "drawn") -> Workload:
    """Seeded circuit phi map: excitable 16-wide channels (0.054) on an
    inhibitory background (0.2), built from (tile x tile) macro-tiles, each
    holding a straight, cross, corner, diode or AND T-junction motif at a
    random rotation.  Every channel runs along a tile's centre line, so
    channels of neighbouring tiles join.  Up to ``ndisks`` r=5 input disks lie
    wholly inside excitable channels at uniformly random steps in [0, steps),
    spaced so that no disk lands where an earlier disk's wave can already
    have passed (``_spaced_disks``; ``disk_order="time"`` keeps the earliest
    candidates, which a long run on a small grid needs: its late candidates
    mostly conflict with early ones).  (Catalysing the phi=0.2 background, or
    re-exciting medium still refractory from an earlier wave, drives forward
    Euler at dt=0.001 into divergence.)"""
    if n % tile:
        raise ValueError("n must be a multiple of the macro-tile size")
    rng = _rng(seed)
    nt = n // tile
    lab = np.zeros((n, n), dtype=np.uint8)
    motifs = rng.integers(0, len(_MOTIFS), size=(nt, nt))
    rots = rng.integers(0, 4, size=(nt, nt))
    for ty in range(nt):
        for tx in range(nt):
            _draw_motif(lab[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile],
                        _MOTIFS[motifs[ty, tx]], int(rots[ty, tx]), rng, tile)
    lut = np.array([PHI_INHIBITORY, PHI_EXCITABLE, DIODE_PHI_GAP, and_phi_gap],
                   dtype=np.float32)
    phi = lut[lab]
    stim = _spaced_disks(rng, lab == _CH, steps, ndisks, disk_order)
    wl = Workload("circuit_%d" % n, n, n, dict(PARAMS_WORKLOAD), phi,
                  _zeros(n, n), _zeros(n, n), stim, steps, seed)
    wl.extra["motif_counts"] = [int((motifs == i).sum()) for i in range(len(_MOTIFS))]
    return wl


# --------------------------------------------------------------------------
# The paper's sanity circuits (Sec. 4), rebuilt from generated geometry
# --------------------------------------------------------------------------

def diode_case(direction: str, params: Optional[Dict[str, float]] = None,
               gap: int = DIODE_GAP, tip: int = DIODE_TIP,
               phi_gap: float = DIODE_PHI_GAP, phi_bg: float = PHI_INHIBITORY,
               phi_act: float = PHI_EXCITABLE, length: int = 160,
               steps: int = 8000, margin: int = 4) -> Workload:
    """A straight 16-wide channel of ``length`` columns along x, cut by a
    diode: a flat channel end, ``gap`` passive columns, then a tip widening
    over ``tip`` columns.  ``direction`` is "flat_to_tip" (wave launched on the
    flat side, the anode of Sec. 4.2) or "tip_to_flat" (launched on the pointed
    side).  The stimulus is a disk at the launching end; the probe cells are
    the far end of the channel (``extra['probe']``: x-range and y-range)."""
    params = dict(PARAMS_WORKLOAD if params is None else params)
    w = CHANNEL_WIDTH
    ny = w + 2 * margin
    nx = length
    blk = np.zeros((ny, nx), dtype=np.uint8)
    blk[margin:margin + w, :] = _CH
    xl = nx // 2 - (gap + tip) // 2
    _draw_diode_gap(blk, margin, xl, gap, tip)
    if direction == "tip_to_flat":
        blk = blk[:, ::-1].copy()
    elif direction != "flat_to_tip":
        raise ValueError(direction)
    lut = np.array([phi_bg, phi_act, phi_gap, phi_gap], dtype=np.float32)
    phi = lut[blk]
    cy = margin + w // 2
    stim = [Stimulus(0, 8, cy, STIM_RADIUS)]
    wl = Workload("diode_%s" % direction, nx, ny, params, phi, _zeros(ny, nx),
                  _zeros(ny, nx), stim, steps, 0)
    wl.extra["probe"] = [nx - 12, nx - 4, margin, margin + w]
    return wl


def and_case(inputs: Tuple[int, int], params: Optional[Dict[str, float]] = None,
             phi_gap: float = AND_PHI_GAP, gap_rows: int = AND_GAP_ROWS,
             phi_bg: float = PHI_INHIBITORY, phi_act: float = PHI_EXCITABLE,
             half_len: int = 64, out_len: int = 48, delay: int = 0,
             steps: int = 9000, margin: int = 4) -> Workload:
    """Coincidence-detector AND gate (Sec. 4.1): a horizontal 16-wide input
    channel, and below its centre a perpendicular 16-wide output channel
    separated from it by ``gap_rows`` passive rows.  ``inputs`` = (left,
    right) selects which channel ends are stimulated; the right input fires
    ``delay`` steps after the left one.  The probe is the bottom of the output
    channel (``extra['probe']``)."""
    params = dict(PARAMS_WORKLOAD if params is None else params)
    w = CHANNEL_WIDTH
    nx = 2 * half_len + w
    ny = margin + w + gap_rows + out_len
    blk = np.zeros((ny, nx), dtype=np.uint8)
    blk[margin:margin + w, :] = _CH
    c0 = half_len
    blk[margin + w:margin + w + gap_rows, c0:c0 + w] = _AND_GAP
    blk[margin + w + gap_rows:, c0:c0 + w] = _CH
    lut = np.array([phi_bg, phi_act, phi_gap, phi_gap], dtype=np.float32)
    phi = lut[blk]
    cy = margin + w // 2
    stim = []
    if inputs[0]:
        stim.append(Stimulus(0, 8, cy, STIM_RADIUS))
    if inputs[1]:
        stim.append(Stimulus(delay if inputs[0] else 0, nx - 9, cy, STIM_RADIUS))
    wl = Workload("and_%d%d" % tuple(inputs), nx, ny, params, phi, _zeros(ny, nx),
                  _zeros(ny, nx), stim, steps, 0)
    wl.extra["probe"] = [c0, c0 + w, ny - 8, ny - 2]
    return wl


# --------------------------------------------------------------------------
# Batched sweep inputs
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SimSpec:
    nx: int
    ny: int
    params: Dict[str, float]
    phi: np.ndarray
    stimuli: List[Stimulus]


def lattice_circuit(nx: int, ny: int, rng: np.random.Generator, phi_act: float,
                    phi_bg: float = PHI_INHIBITORY, spacing: int = 96) -> np.ndarray:
    """A lattice of 16-wide channels (``phi_act``) on ``phi_bg`` with a seeded
    offset and spacing; some lattice segments carry a diode cut or an AND gap."""
    w = CHANNEL_WIDTH
    lab = np.zeros((ny, nx), dtype=np.uint8)
    oy = int(rng.integers(0, max(1, min(spacing, ny - w))))
    ox = int(rng.integers(0, max(1, min(spacing, nx - w))))
    for y in range(oy % spacing, ny - w + 1, spacing):
        lab[y:y + w, :] = _CH
    for x in range(ox % spacing, nx - w + 1, spacing):
        lab[:, x:x + w] = _CH
    if not lab.any():
        y = (ny - w) // 2 if ny > w else 0
        lab[y:y + min(w, ny), :] = _CH
    return np.where(lab == _CH, np.float32(phi_act), np.float32(phi_bg)).astype(np.float32)


def batch_sweep(count: int = 512, seed: int = 1004, smin: int = 64, smax: int = 1024,
                steps: int = 5000) -> Tuple[List[SimSpec], int]:
    """``count`` independent simulations: each side round(smin*(smax/smin)^U),
    U ~ U[0,1) drawn independently; eps ~ U[0.02, 0.03], phi_excitable ~
    U[0.04, 0.08], background 0.2, a channel lattice scaled to the grid, and
    1-4 r=5 disks wholly inside channels at t=0, DISK_MARGIN apart."""
    rng = _rng(seed)
    sims: List[SimSpec] = []
    ratio = smax / smin
    for _ in range(count):
        nx = int(round(smin * ratio ** rng.random()))
        ny = int(round(smin * ratio ** rng.random()))
        eps = float(rng.uniform(0.02, 0.03))
        pa = float(rng.uniform(0.04, 0.08))
        p = dict(PARAMS_WORKLOAD)
        p["eps"] = eps
        spacing = int(max(32, min(nx, ny) // 3))
        phi = lattice_circuit(nx, ny, rng, pa, spacing=spacing)
        ys, xs = np.nonzero(_disk_fits(phi == np.float32(pa), STIM_RADIUS))
        k = int(rng.integers(1, 5))
        pick = rng.integers(0, ys.size, size=4 * k)
        stim = []
        for i in pick:               # keep disks DISK_MARGIN apart (fewer if they do not fit)
            if all(np.hypot(int(xs[i]) - d.cx, int(ys[i]) - d.cy) >= DISK_MARGIN for d in stim):
                stim.append(Stimulus(0, int(xs[i]), int(ys[i]), STIM_RADIUS))
                if len(stim) == k:
                    break
        sims.append(SimSpec(nx, ny, p, phi, stim))
    return sims, steps


# --------------------------------------------------------------------------
# Small synthetic fields for tests
# --------------------------------------------------------------------------

def random_state(nx: int, ny: int, seed: int, umax: float = 1.0, vmax: float = 0.05,
                 phi_lo: float = 0.04, phi_hi: float = 0.1
                 ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Random (u, v, phi) fields with u in [0, umax), v in [0, vmax), phi in
    [phi_lo, phi_hi) -- states a running simulation can reach."""
    rng = _rng(seed)
    u = (rng.random((ny, nx)) * umax).astype(np.float32)
    v = (rng.random((ny, nx)) * vmax).astype(np.float32)
    phi = (phi_lo + rng.random((ny, nx)) * (phi_hi - phi_lo)).astype(np.float32)
    return u, v, phi


def random_disks(nx: int, ny: int, count: int, seed: int, rmax: int = 6
                 ) -> List[Stimulus]:
    rng = _rng(seed)
    return [Stimulus(0, int(rng.integers(0, nx)), int(rng.integers(0, ny)),
                     int(rng.integers(0, rmax + 1))) for _ in range(count)]


def pitch_for(nx: int, align: int = 64) -> int:
    """Row pitch (elements) used for device planes: a multiple of 64."""
    return (nx + align - 1) // align * align


__all__: Sequence[str] = [
    "PARAMS_TABLE1", "PARAMS_WORKLOAD", "PHI_ACTIVE_TABLE1", "PHI_PASSIVE_TABLE1",
    "PHI_EXCITABLE", "PHI_INHIBITORY", "Stimulus", "Workload", "SimSpec",
    "single_disk", "uniform_random_phi", "circuit", "diode_case", "and_case",
    "batch_sweep", "random_state", "random_disks", "pitch_for", "lattice_circuit",
    "spacing_ok",
]
