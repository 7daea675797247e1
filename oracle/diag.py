"""Oracle-side post-processing of force histories (FP64, plain NumPy).

TEST INFRASTRUCTURE: computes the paper's force coefficients and Strouhal
number from the oracle's force records, independently of the HIP library's own
diagnostics.

- C_d = 2 F_d / (rho U^2 D), C_l = 2 F_l / (rho U^2 D)  (paper Sec. 3), with the
  force taken on the body (so C_d > 0 for a body held in a +x stream).
- St = f_q D / U (paper Sec. 3) with f_q from the lift signal: the mean period
  between upward crossings of C_l - mean(C_l), crossing times linearly
  interpolated, over the given window.
- The steady-wake quantities of Sec. 3.2's low-Re table (recirculation length
  and separation angle), read from the oracle's fields; defined below.
"""
from __future__ import annotations

import numpy as np


def coefficients(force_xy: np.ndarray, u: float, length: float, rho: float = 1.0):
    f = np.asarray(force_xy, dtype=np.float64)
    q = 0.5 * rho * u * u * length
    return f[..., 0] / q, f[..., 1] / q


def upward_crossing_times(signal: np.ndarray, dt: float = 1.0) -> np.ndarray:
    s = np.asarray(signal, dtype=np.float64)
    s = s - s.mean()
    out = []
    for k in range(len(s) - 1):
        if s[k] < 0.0 <= s[k + 1]:
            frac = -s[k] / (s[k + 1] - s[k])
            out.append((k + frac) * dt)
    return np.array(out)


def strouhal(cl: np.ndarray, dt: float, u: float, length: float) -> float:
    t = upward_crossing_times(cl, dt)
    if len(t) < 3:
        return float("nan")
    period = (t[-1] - t[0]) / (len(t) - 1)
    return length / (period * u)


def shedding_summary(force_xy: np.ndarray, dt: float, u: float, length: float) -> dict:
    cd, cl = coefficients(force_xy, u, length)
    return {
        "cd_mean": float(cd.mean()),
        "cd_amp": float((cd.max() - cd.min()) / 2.0),
        "cl_amp": float((cl.max() - cl.min()) / 2.0),
        "st": strouhal(cl, dt, u, length),
    }


# ------------------------------------------------------------ steady wakes --
# Sec. 3.2, Table low-Re: the recirculation length L_s (from the rear of the
# cylinder to the end of the reversed-flow bubble on the wake axis, over D) and
# the separation angle theta_s (from the rear stagnation point to where the
# boundary layer leaves the body). The grid quantities they are read from:
#  - L_s: u_x on the axis y = c_y (linear in y between the two rows around it),
#    from the first node behind x = c_x + R to the first sign change from
#    negative to non-negative, located by linear interpolation between nodes;
#    no reversed flow at that first node gives 0;
#  - theta_s: the tangential velocity on the circle r = R + offset (bilinear in
#    the grid), positive away from the rear stagnation point; theta_s is the
#    first angle past `skip_deg` where it turns from positive to non-positive,
#    averaged over the upper and lower halves (0 if the flow there is attached).


def _axis_value(ux: np.ndarray, i: int, cy: float) -> float:
    j = int(np.floor(cy))
    w = cy - j
    if w == 0.0:
        return float(ux[j, i])
    return float((1.0 - w) * ux[j, i] + w * ux[j + 1, i])


def wake_length(ux: np.ndarray, cx: float, cy: float, radius: float) -> float:
    """L_s / D of the steady wake behind a cylinder in a +x stream."""
    nx = ux.shape[1]
    rear = cx + radius
    i = int(np.floor(rear)) + 1
    if i >= nx - 1 or _axis_value(ux, i, cy) >= 0.0:
        return 0.0
    prev = _axis_value(ux, i, cy)
    while i + 1 < nx:
        nxt = _axis_value(ux, i + 1, cy)
        if nxt >= 0.0:
            x_end = i + prev / (prev - nxt)
            return (x_end - rear) / (2.0 * radius)
        prev = nxt
        i += 1
    return float("nan")


def _bilinear_at(field: np.ndarray, x: float, y: float) -> float:
    i0 = int(np.floor(x))
    j0 = int(np.floor(y))
    fx = x - i0
    fy = y - j0
    top = field[j0 + 1, i0] + fx * (field[j0 + 1, i0 + 1] - field[j0 + 1, i0])
    bot = field[j0, i0] + fx * (field[j0, i0 + 1] - field[j0, i0])
    return float(bot + fy * (top - bot))


def _tangential(ux, uy, cx, cy, r, th, side):
    """Velocity along the circle in the direction of growing angle th, measured
    from the rear (+x) on the upper (side = +1) or lower (-1) half."""
    x = cx + r * np.cos(th)
    y = cy + side * r * np.sin(th)
    vx = _bilinear_at(ux, x, y)
    vy = _bilinear_at(uy, x, y)
    # unit tangent of (cos th, side sin th) in th: (-sin th, side cos th)
    return -np.sin(th) * vx + side * np.cos(th) * vy


def separation_angle(ux: np.ndarray, uy: np.ndarray, cx: float, cy: float, radius: float,
                     offset: float = 1.5, skip_deg: float = 3.0, coarse_deg: float = 0.25) -> float:
    """theta_s in degrees: scan the circle in steps of coarse_deg from skip_deg,
    then bisect the first bracket where the tangential velocity leaves positive."""
    r = radius + offset
    found = []
    for side in (1.0, -1.0):
        a = np.radians(skip_deg)
        va = _tangential(ux, uy, cx, cy, r, a, side)
        if va <= 0.0:
            return 0.0
        step = np.radians(coarse_deg)
        bracket = None
        while a < np.pi:
            b = min(a + step, np.pi)
            vb = _tangential(ux, uy, cx, cy, r, b, side)
            if vb <= 0.0:
                bracket = (a, b)
                break
            a = b
        if bracket is None:
            return 0.0
        lo, hi = bracket
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            if _tangential(ux, uy, cx, cy, r, mid, side) > 0.0:
                lo = mid
            else:
                hi = mid
        found.append(np.degrees(0.5 * (lo + hi)))
    return float(0.5 * (found[0] + found[1]))
