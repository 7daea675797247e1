"""Post-processing of solver output (host, FP64): force coefficients, Strouhal
number, and the steady-wake quantities of the low-Reynolds cylinder cases.

- C_d = 2 F_x / (rho U^2 L), C_l = 2 F_y / (rho U^2 L) with the force on the body
  (Sec. 3; L the diameter or chord, rho the reference density 1).
- St = f L / U with f from the lift signal: mean period between upward crossings
  of C_l - mean(C_l), crossing times linearly interpolated.
- Recirculation length L_s / D (Sec. 3.2, low-Re table): from the rear of the
  cylinder to the point on the wake centreline where the streamwise velocity
  turns positive again, linearly interpolated between nodes.
- Separation angle theta_s (same table): on a circle just outside the body,
  the angle from the rear stagnation point at which the tangential velocity
  changes sign, bilinearly sampled, averaged over the upper and lower halves.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np


def force_coefficients(force_xy: np.ndarray, u: float, length: float, rho: float = 1.0):
    f = np.asarray(force_xy, dtype=np.float64)
    q = 0.5 * rho * u * u * length
    return f[..., 0] / q, f[..., 1] / q


def strouhal(cl: np.ndarray, dt: float, u: float, length: float) -> float:
    s = np.asarray(cl, dtype=np.float64)
    s = s - s.mean()
    k = np.nonzero((s[:-1] < 0.0) & (s[1:] >= 0.0))[0]
    if len(k) < 3:
        return float("nan")
    t = (k + (-s[k] / (s[k + 1] - s[k]))) * dt
    period = (t[-1] - t[0]) / (len(t) - 1)
    return length / (period * u)


def shedding(force_xy: np.ndarray, dt: float, u: float, length: float) -> Dict[str, float]:
    """Mean drag, drag and lift amplitudes ((max - min) / 2) and St of a record
    window (records dt steps apart)."""
    cd, cl = force_coefficients(force_xy, u, length)
    return {"cd_mean": float(cd.mean()), "cd_amp": float((cd.max() - cd.min()) / 2.0),
            "cl_amp": float((cl.max() - cl.min()) / 2.0), "st": strouhal(cl, dt, u, length)}


def _bilinear(f: np.ndarray, x: float, y: float) -> float:
    i, j = int(math.floor(x)), int(math.floor(y))
    a, b = x - i, y - j
    return float((1 - a) * (1 - b) * f[j, i] + a * (1 - b) * f[j, i + 1]
                 + (1 - a) * b * f[j + 1, i] + a * b * f[j + 1, i + 1])


def recirculation_length(ux: np.ndarray, cx: float, cy: float, radius: float) -> float:
    """L_s / D behind a cylinder of the given centre and radius in a +x stream:
    walk the centreline row (interpolated between the two rows around cy) from
    the rear surface to the first node with u_x > 0 after a reversed region."""
    ny, nx = ux.shape
    j0 = int(math.floor(cy))
    w = cy - j0
    line = (1 - w) * ux[j0] + w * ux[j0 + 1] if w > 0 else ux[j0].copy()
    start = int(math.floor(cx + radius)) + 1
    if start >= nx - 1 or line[start] >= 0.0:
        return 0.0
    for i in range(start, nx - 1):
        if line[i] < 0.0 <= line[i + 1]:
            x0 = i + (-line[i]) / (line[i + 1] - line[i])
            return (x0 - (cx + radius)) / (2.0 * radius)
    return float("nan")


def separation_angle(ux: np.ndarray, uy: np.ndarray, cx: float, cy: float, radius: float,
                     offset: float = 1.5, samples: int = 3600, skip_deg: float = 3.0) -> float:
    """theta_s in degrees, measured from the rear stagnation point (+x side) to
    where the tangential velocity on the circle r = radius + offset first turns
    from positive (bubble) to negative (attached flow); mean of the upper and
    lower halves. The first skip_deg degrees are skipped: at the stagnation
    point itself the tangential velocity vanishes and its sign is noise."""
    r = radius + offset
    th = np.linspace(math.radians(skip_deg), math.pi, samples)
    angles = []
    for sgn in (1.0, -1.0):
        ut = []
        for t in th:
            x, y = cx + r * math.cos(t), cy + sgn * r * math.sin(t)
            vx, vy = _bilinear(ux, x, y), _bilinear(uy, x, y)
            # component along the direction of increasing t, (-sin t, sgn cos t)
            ut.append(-math.sin(t) * vx + sgn * math.cos(t) * vy)
        ut = np.array(ut)
        # inside the recirculation bubble the near-wall flow runs away from the
        # rear stagnation point (u_t > 0); the attached flow runs toward it
        if ut[0] <= 0.0:
            return 0.0                      # no reversed flow behind the body
        k = np.nonzero((ut[:-1] > 0.0) & (ut[1:] <= 0.0))[0]
        if len(k) == 0:
            return 0.0
        k = k[0]
        t0 = th[k] + (th[k + 1] - th[k]) * (-ut[k]) / (ut[k + 1] - ut[k])
        angles.append(math.degrees(t0))
    return float(np.mean(angles))


def steady_wake(fields: Dict[str, np.ndarray], cx: float, cy: float, radius: float) -> Tuple[float, float]:
    """(L_s / D, theta_s in degrees) of a steady cylinder wake."""
    return (recirculation_length(fields["ux"], cx, cy, radius),
            separation_angle(fields["ux"], fields["uy"], cx, cy, radius))
