"""Pins of the oracle-side post-processing (``oracle/diag.py``) on signals and
fields whose answers are fixed in closed form, independently of the code:

- force coefficients (Sec. 3): C = 2 F / (rho U^2 D) of a known force;
- the Strouhal number St = f D / U (Sec. 3) of sinusoidal lift signals with
  known, non-integer periods, an offset mean and a phase, sampled every dt
  steps; upward-crossing times of a signal whose crossings are known exactly;
- mean and (max - min)/2 amplitudes of signals sampled exactly at their extrema;
- the recirculation length of Sec. 3.2 on a field linear in x and y (so that
  the interpolation between rows and nodes is exact), off-row centre included;
- the separation angle of Sec. 3.2 on linear fields (bilinear sampling is then
  exact): a symmetric one with a closed-form angle, and an asymmetric one whose
  two half-angles come from a root finder.

Each check takes the module as an argument, so ``test_oracle_diag_mutations``
can run the same checks against copies with planted mistakes.
"""
import math

import numpy as np
from scipy.optimize import brentq


def check_coefficients(d):
    u, length = 0.05, 40.0
    q = 0.5 * 1.0 * u * u * length
    f = np.array([[1.25 * q, -0.5 * q], [2.0 * q, 0.125 * q]])
    cd, cl = d.coefficients(f, u, length)
    assert np.allclose(cd, [1.25, 2.0], rtol=1e-15, atol=0) and np.allclose(cl, [-0.5, 0.125], rtol=1e-15, atol=0)
    cd, _ = d.coefficients(f, u, length, rho=2.0)
    assert np.allclose(cd, [0.625, 1.0], rtol=1e-15, atol=0)


def check_crossing_times(d):
    # +-1 alternating: mean 0, upward crossings half-way between samples 2k+1 and 2k+2
    s = np.array([1.0, -1.0] * 6)
    t = d.upward_crossing_times(s, dt=3.0)
    assert np.allclose(t, 3.0 * (np.arange(1, 11, 2) + 0.5), rtol=0, atol=1e-12)
    # mean 0, one upward crossing 3/4 of the way from sample 0 to sample 1
    t = d.upward_crossing_times(np.array([-3.0, 1.0, 1.0, 1.0]), dt=2.0)
    assert len(t) == 1 and abs(t[0] - 1.5) < 1e-15
    # the mean is removed first: the same signal lifted by 5 crosses at the same time
    t = d.upward_crossing_times(np.array([2.0, 6.0, 6.0, 6.0]), dt=2.0)
    assert len(t) == 1 and abs(t[0] - 1.5) < 1e-15


def check_strouhal(d):
    u, length = 0.05, 40.0
    for period, dt, phase, mean in [(23.7, 1.0, 0.3, 0.2), (187.3, 5.0, 1.9, -0.4), (61.15, 2.0, 4.0, 0.0)]:
        n = int(40 * period / dt)
        t = np.arange(n) * dt
        cl = mean + 0.3 * np.sin(2.0 * math.pi * t / period + phase)
        st = d.strouhal(cl, dt, u, length)
        assert abs(st - length / (period * u)) <= 1e-4 * st, (period, dt, st)
    assert math.isnan(d.strouhal(np.linspace(-1.0, 1.0, 50), 1.0, u, length))   # one crossing only


def check_summary(d):
    u, length = 0.05, 40.0
    q = 0.5 * u * u * length
    k = np.arange(1000)
    cd = 1.3 + 0.02 * np.cos(2.0 * math.pi * k / 20.0)       # 20 samples per period, peaks sampled
    cl = 0.3 * np.sin(2.0 * math.pi * k / 40.0)              # extrema at k = 10, 30 (mod 40)
    s = d.shedding_summary(np.stack([q * cd, q * cl], -1), 4.0, u, length)
    assert abs(s["cd_mean"] - 1.3) < 1e-12
    assert abs(s["cd_amp"] - 0.02) < 1e-12
    assert abs(s["cl_amp"] - 0.3) < 1e-12
    assert abs(s["st"] - length / (160.0 * u)) < 1e-6 * s["st"]


def _linear_wake(nx, ny, cx, cy, x_end):
    """u_x = (x - x_end) + 0.5 (y - cy): on the axis y = cy it turns positive at
    x_end; linear in both coordinates, so interpolation is exact."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return (x - x_end) + 0.5 * (y - cy)


def check_wake_length(d):
    for cx, cy, radius, ls in [(60.0, 50.0, 10.0, 23.7), (60.3, 50.4, 9.5, 11.25), (40.7, 31.6, 6.0, 0.35)]:
        x_end = cx + radius + ls
        ux = _linear_wake(200, 101, cx, cy, x_end)
        if math.floor(cx + radius) + 1 >= x_end:
            continue
        got = d.wake_length(ux, cx, cy, radius)
        assert abs(got - ls / (2.0 * radius)) < 1e-12, (cx, cy, got)
    # no reversed flow right behind the body: no bubble
    assert d.wake_length(np.ones((40, 80)), 20.0, 20.0, 5.0) == 0.0
    ux = _linear_wake(80, 40, 20.0, 20.0, 24.5)                 # bubble ends before the first node
    assert d.wake_length(ux, 20.0, 20.0, 5.0) == 0.0


def _linear_field(nx, ny, cx, cy, a, c=0.0):
    """u_x = a - (x - cx), u_y = (y - cy) + c. On the circle of radius r about the
    centre the tangential velocity (growing angle th from the rear, half `side`)
    is -sin th (a - 2 r cos th) + side c cos th."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return a - (x - cx), (y - cy) + c


def check_separation_angle(d):
    cx, cy, radius, offset = 100.3, 60.6, 12.0, 1.5
    r = radius + offset
    for theta in (43.0, 52.9, 71.0):
        a = 2.0 * r * math.cos(math.radians(theta))             # u_t = 0 at cos th = a / (2 r)
        ux, uy = _linear_field(220, 130, cx, cy, a)
        got = d.separation_angle(ux, uy, cx, cy, radius, offset=offset)
        assert abs(got - theta) < 1e-6, (theta, got)
    # asymmetric: the two halves separate at different angles; theta_s is their mean
    a, c = 2.0 * r * math.cos(math.radians(50.0)), 0.3
    ux, uy = _linear_field(220, 130, cx, cy, a, c)
    halves = []
    for side in (1.0, -1.0):
        ut = lambda th, s=side: -math.sin(th) * (a - 2.0 * r * math.cos(th)) + s * c * math.cos(th)  # noqa: E731
        assert ut(math.radians(3.0)) > 0.0
        grid = np.radians(np.arange(3.0, 180.0, 0.5))
        k = next(i for i in range(len(grid) - 1) if ut(grid[i + 1]) <= 0.0)
        halves.append(math.degrees(brentq(ut, grid[k], grid[k + 1], xtol=1e-14)))
    assert abs(halves[0] - halves[1]) > 1.0
    got = d.separation_angle(ux, uy, cx, cy, radius, offset=offset)
    assert abs(got - 0.5 * (halves[0] + halves[1])) < 1e-6, (got, halves)
    # attached flow (u_t <= 0 right behind the body) has no separation
    ux, uy = _linear_field(220, 130, cx, cy, 3.0 * r)
    assert d.separation_angle(ux, uy, cx, cy, radius, offset=offset) == 0.0


CHECKS = [check_coefficients, check_crossing_times, check_strouhal, check_summary, check_wake_length,
          check_separation_angle]


def test_coefficients():
    from oracle import diag
    check_coefficients(diag)


def test_crossing_times():
    from oracle import diag
    check_crossing_times(diag)


def test_strouhal():
    from oracle import diag
    check_strouhal(diag)


def test_summary():
    from oracle import diag
    check_summary(diag)


def test_wake_length():
    from oracle import diag
    check_wake_length(diag)


def test_separation_angle():
    from oracle import diag
    check_separation_angle(diag)
