"""Drawing tools for excitability maps, after the app's editor (Sec. 3).

The app draws freehand strokes and straight lines either of substrate (phi)
or of catalytic stimulation (u := 1), on a 400 x 300 grid, with:

  * a snap-line option that restricts a straight line's direction to
    multiples of 15 degrees;
  * line-width presets: permeable 2, semi-permeable 3, impermeable 8 pixels;
  * background presets: "filled" (excitable substrate everywhere; the user
    removes it by drawing passive lines) or "empty" (passive everywhere; the
    user adds excitable substrate).

Rasterisation (not specified by the paper; this module's choice): cell
(x, y) is painted when its centre (x + 0.5, y + 0.5) lies closer than w/2 to
the stroke's centre line (round caps).  A stroke between integer cell
coordinates runs through cell centres for odd widths and along cell corners
for even widths, so horizontal and vertical lines are exactly w cells wide.
Only geometry lives here: no arithmetic of the model.
"""
from __future__ import annotations

import math
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

from .inputs import PHI_ACTIVE_TABLE1, PHI_PASSIVE_TABLE1, Stimulus

APP_GRID = (400, 300)                 # the app's simulation grid, nx x ny (Sec. 3)
SNAP_DEG = 15                         # snap-line angle step (Sec. 3)
WIDTH_PRESETS = {"permeable": 2, "semi-permeable": 3, "impermeable": 8}


def snap_angle(deg: float) -> float:
    """Nearest multiple of 15 degrees."""
    return SNAP_DEG * round(deg / SNAP_DEG)


def snapped_end(p0: Sequence[float], p1: Sequence[float]) -> Tuple[float, float]:
    """End point of a snap line from p0 towards p1: same length, direction
    rounded to a multiple of 15 degrees."""
    dx, dy = p1[0] - p0[0], p1[1] - p0[1]
    length = math.hypot(dx, dy)
    a = math.radians(snap_angle(math.degrees(math.atan2(dy, dx))))
    return (p0[0] + length * math.cos(a), p0[1] + length * math.sin(a))


def _width(width) -> int:
    return WIDTH_PRESETS[width] if isinstance(width, str) else int(width)


def stroke_mask(nx: int, ny: int, points: Sequence[Sequence[float]], width) -> np.ndarray:
    """Boolean (ny, nx) mask of a polyline of `width` (pixels or a preset
    name) through `points` (cell coordinates, x then y)."""
    w = _width(width)
    if w < 1:
        raise ValueError("line width must be >= 1")
    off = 0.5 if w % 2 else 0.0
    pts = [(float(p[0]) + off, float(p[1]) + off) for p in points]
    mask = np.zeros((ny, nx), dtype=bool)
    half = w / 2.0
    if len(pts) == 1:
        pts = pts * 2
    for (ax, ay), (bx, by) in zip(pts[:-1], pts[1:]):
        x0 = max(0, int(math.floor(min(ax, bx) - half)))
        x1 = min(nx, int(math.ceil(max(ax, bx) + half)) + 1)
        y0 = max(0, int(math.floor(min(ay, by) - half)))
        y1 = min(ny, int(math.ceil(max(ay, by) + half)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        cy, cx = np.mgrid[y0:y1, x0:x1]
        px, py = cx + 0.5, cy + 0.5
        vx, vy = bx - ax, by - ay
        ll = vx * vx + vy * vy
        t = np.zeros_like(px) if ll == 0 else np.clip(((px - ax) * vx + (py - ay) * vy) / ll,
                                                      0.0, 1.0)
        d2 = (px - ax - t * vx) ** 2 + (py - ay - t * vy) ** 2
        mask[y0:y1, x0:x1] |= d2 < half * half
    return mask


class Canvas:
    """An excitability map being drawn, plus the stimulation strokes drawn
    on it.  `background`: "filled" or "empty" (Sec. 3 presets)."""

    def __init__(self, nx: int = APP_GRID[0], ny: int = APP_GRID[1], background: str = "empty",
                 phi_active: float = PHI_ACTIVE_TABLE1, phi_passive: float = PHI_PASSIVE_TABLE1):
        if background not in ("filled", "empty"):
            raise ValueError("background must be 'filled' or 'empty'")
        self.nx, self.ny = int(nx), int(ny)
        self.phi_active, self.phi_passive = float(phi_active), float(phi_passive)
        fill = self.phi_active if background == "filled" else self.phi_passive
        self.phi = np.full((self.ny, self.nx), fill, dtype=np.float32)
        self.stim = np.zeros((self.ny, self.nx), dtype=bool)

    def _paint(self, mask: np.ndarray, what: str) -> None:
        if what == "passive":
            self.phi[mask] = np.float32(self.phi_passive)
        elif what == "active":
            self.phi[mask] = np.float32(self.phi_active)
        elif what == "stimulus":
            self.stim |= mask
        else:
            raise ValueError("what must be 'passive', 'active' or 'stimulus'")

    def line(self, p0, p1, width, what: str = "passive", snap: bool = False) -> np.ndarray:
        """Straight line from p0 to p1 (cell coordinates); with snap=True its
        direction is rounded to a multiple of 15 degrees.  Returns its mask."""
        end = snapped_end(p0, p1) if snap else p1
        m = stroke_mask(self.nx, self.ny, [p0, end], width)
        self._paint(m, what)
        return m

    def freehand(self, points: Iterable[Sequence[float]], width,
                 what: str = "passive") -> np.ndarray:
        m = stroke_mask(self.nx, self.ny, list(points), width)
        self._paint(m, what)
        return m

    def stimulus_disks(self, step: int = 0, r: int = 0) -> List[Stimulus]:
        """The drawn stimulation as radius-r disks (r = 0: single cells) at
        `step`, for the stepper's stimulate call."""
        ys, xs = np.nonzero(self.stim)
        return [Stimulus(int(step), int(x), int(y), int(r)) for x, y in zip(xs, ys)]

    def stimulated_u(self, u: Optional[np.ndarray] = None) -> np.ndarray:
        """u with the drawn stimulation applied (u := 1 on stroke cells)."""
        out = np.zeros((self.ny, self.nx), np.float32) if u is None else np.array(u, np.float32)
        out[self.stim] = 1.0
        return out
