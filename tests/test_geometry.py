"""Drawing tools (Sec. 3): exact preset widths, 15-degree snap lines,
background presets, strokes, and the permeable / impermeable line presets'
effect on a planar wave in the FP64 oracle at Table 1 parameters."""
import math

import numpy as np
import pytest

import oracle
from paper_1901_06535_amd import geometry as G
from paper_1901_06535_amd import inputs


@pytest.mark.parametrize("w", range(1, 9))
def test_axis_aligned_lines_are_exactly_w_cells_wide(w):
    c = G.Canvas(60, 50, background="filled")
    m = c.line((10, 20), (40, 20), w)                  # horizontal
    cols = m[:, 15:35].sum(axis=0)
    assert (cols == w).all()
    m2 = G.stroke_mask(60, 50, [(25, 5), (25, 45)], w)  # vertical
    assert (m2[10:40, :].sum(axis=1) == w).all()
    assert (c.phi[m] == np.float32(inputs.PHI_PASSIVE_TABLE1)).all()
    assert (c.phi[~m] == np.float32(inputs.PHI_ACTIVE_TABLE1)).all()


def test_presets_and_backgrounds():
    assert G.WIDTH_PRESETS == {"permeable": 2, "semi-permeable": 3, "impermeable": 8}
    assert G.APP_GRID == (400, 300)
    e = G.Canvas(background="empty")
    assert e.phi.shape == (300, 400) and (e.phi == np.float32(inputs.PHI_PASSIVE_TABLE1)).all()
    m = e.line((50, 100), (350, 100), "impermeable", what="active")
    assert (m[:, 100:300].sum(axis=0) == 8).all()
    assert (e.phi[m] == np.float32(inputs.PHI_ACTIVE_TABLE1)).all()
    with pytest.raises(ValueError):
        G.Canvas(background="grey")


@pytest.mark.parametrize("target,expect", [((100, 3), 0), ((70, 40), 30), ((-50, 48), 135),
                                           ((3, -90), -90), ((80, 22), 15)])
def test_snap_line_direction_is_a_multiple_of_15_degrees(target, expect):
    p0 = (0.0, 0.0)
    end = G.snapped_end(p0, target)
    ang = math.degrees(math.atan2(end[1], end[0]))
    assert abs(ang - expect) < 1e-9 or abs(abs(ang - expect) - 360) < 1e-9
    assert abs(math.hypot(*end) - math.hypot(*target)) < 1e-9
    assert G.snap_angle(7.4) == 0 and G.snap_angle(7.6) == 15 and G.snap_angle(-22) == -15


def test_snap_line_rasterises_along_the_snapped_direction():
    c = G.Canvas(200, 200)
    m = c.line((20, 20), (170, 95), 3, snap=True)        # 26.6 deg -> 30 deg
    ys, xs = np.nonzero(m)
    slope = np.polyfit(xs + 0.5, ys + 0.5, 1)[0]
    assert abs(math.degrees(math.atan(slope)) - 30.0) < 0.5


def test_freehand_stroke_covers_its_polyline_and_stimulus_cells():
    c = G.Canvas(80, 60)
    pts = [(5, 5), (30, 10), (40, 40), (70, 50)]
    m = c.freehand(pts, 4, what="stimulus")
    for (ax, ay), (bx, by) in zip(pts[:-1], pts[1:]):
        for t in np.linspace(0, 1, 50):
            x, y = ax + t * (bx - ax), ay + t * (by - ay)
            assert m[int(math.floor(y)), int(math.floor(x))]
    assert (c.phi == np.float32(inputs.PHI_PASSIVE_TABLE1)).all()   # stimulus leaves phi
    u = c.stimulated_u()
    assert (u[m] == 1.0).all() and (u[~m] == 0.0).all()
    disks = c.stimulus_disks(step=7)
    assert len(disks) == int(m.sum()) and all(d.step == 7 and d.r == 0 for d in disks)


def _wave_through_line(width, nx=110, ny=40, x_line=50, x_probe=95, steps=9000):
    c = G.Canvas(nx, ny, background="filled")
    if width:
        c.line((x_line, -10), (x_line, ny + 10), width)
    c.line((3, -5), (3, ny + 5), 4, what="stimulus")
    u0 = c.stimulated_u()
    r = oracle.Run(u0, np.zeros_like(u0), c.phi, inputs.PARAMS_TABLE1, track_arrival=True)
    r.advance(steps)
    far = r.arrival[:, x_probe]
    return int(far.min()) if (far < oracle.NEVER).any() else None


def test_permeable_line_slows_and_impermeable_line_stops_a_planar_wave():
    """At Table 1 parameters (eps 0.0243, D_u 0.45, phi 0.054 / 0.0975), a
    planar wave crosses a 2-pixel passive line later than open medium, and an
    8-pixel line stops it: the paper's permeable and impermeable presets.
    (3 pixels also stops it here, at every approach angle probed: the
    semi-permeable preset's behaviour depends on a discretisation the paper
    does not give, so it is not pinned.)"""
    t_open = _wave_through_line(0)
    t_perm = _wave_through_line(G.WIDTH_PRESETS["permeable"])
    t_imp = _wave_through_line(G.WIDTH_PRESETS["impermeable"])
    assert t_open is not None and t_perm is not None
    assert t_perm > t_open + 20
    assert t_imp is None
