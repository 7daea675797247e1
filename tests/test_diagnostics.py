"""Host post-processing (paper_1901_08766_amd.diagnostics) on fields and
signals whose answers are known in closed form."""
import math

import numpy as np

from paper_1901_08766_amd import diagnostics as dg


def test_coefficients_and_strouhal_of_a_sinusoid():
    u, length, dt = 0.05, 40.0, 10.0
    q = 0.5 * u * u * length
    t = np.arange(20000) * dt
    period = 4700.0                                   # steps
    f = np.stack([q * (1.3 + 0.01 * np.cos(4 * math.pi * t / period)), q * 0.3 * np.sin(2 * math.pi * t / period)], -1)
    s = dg.shedding(f, dt, u, length)
    assert abs(s["cd_mean"] - 1.3) < 1e-3 and abs(s["cd_amp"] - 0.01) < 1e-4 and abs(s["cl_amp"] - 0.3) < 1e-4
    assert abs(s["st"] - length / (period * u)) < 1e-4 * s["st"]


def _wake_field(nx, ny, cx, cy, radius, x_reattach, theta_s):
    """u_x on the centreline reverses between the body and x_reattach; near the
    body the tangential velocity changes sign at theta_s (from the rear)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = x - cx, y - cy
    r = np.hypot(dx, dy)
    t = np.arctan2(np.abs(dy), dx)                     # 0 at the rear, pi at the front
    sgn = np.where(dy >= 0, 1.0, -1.0)
    f = (theta_s - t)                                 # > 0 inside the bubble
    tx, ty = -np.sin(t), sgn * np.cos(t)              # direction of increasing t
    ux, uy = f * tx, f * ty
    band = np.abs(dy) < 3.0
    ux = np.where(band & (dx > radius), (dx - radius) - (x_reattach - cx - radius), ux)
    return ux, uy


def test_recirculation_length_and_separation_angle():
    cx, cy, radius = 60.3, 50.4, 10.0
    x_re = cx + radius + 23.7                         # L_s = 23.7 / 20
    theta = math.radians(47.0)
    ux, uy = _wake_field(200, 101, cx, cy, radius, x_re, theta)
    assert abs(dg.recirculation_length(ux, cx, cy, radius) - 23.7 / 20.0) < 1e-9
    for off in (1.5, 6.0):
        assert abs(dg.separation_angle(ux, uy, cx, cy, radius, offset=off) - 47.0) < 0.5
    # attached flow everywhere: no separation
    assert dg.separation_angle(-np.abs(ux) * 0 + 1.0, np.zeros_like(uy), cx, cy, radius) == 0.0


def test_no_bubble_gives_zero_length():
    ux = np.ones((40, 80))
    assert dg.recirculation_length(ux, 20.0, 20.0, 5.0) == 0.0
