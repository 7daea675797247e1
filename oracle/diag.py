"""Oracle-side post-processing of force histories (FP64, plain NumPy).

TEST INFRASTRUCTURE: computes the paper's force coefficients and Strouhal
number from the oracle's force records, independently of the HIP library's own
diagnostics.

- C_d = 2 F_d / (rho U^2 D), C_l = 2 F_l / (rho U^2 D)  (paper Sec. 3), with the
  force taken on the body (so C_d > 0 for a body held in a +x stream).
- St = f_q D / U (paper Sec. 3) with f_q from the lift signal: the mean period
  between upward crossings of C_l - mean(C_l), crossing times linearly
  interpolated, over the given window.
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
