"""Exact rational-arithmetic evaluation of the TRT-LBM-VP step on tiny grids.

An independent re-statement of the paper's scheme (Sec. 2) used only to pin the
FP64 oracle: every quantity is a ``fractions.Fraction``, so the result is the
scheme's exact value for the given (exactly representable) inputs. It is written
from the equations, not from the oracle's source: the lattice vectors come from
the angle formula of eq. (D2Q9), the opposite direction is found by search, and
the collision is assembled from its definition as f + Omega + forcing.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from typing import Dict, List, Sequence, Tuple

CS2 = Fr(1, 3)  # c_s^2, c_s = 1/sqrt(3)


def velocities() -> List[Tuple[int, int]]:
    """eq. (D2Q9): rest, then (cos t, sin t) with t = (a-1) pi/2 for a = 1..4,
    then sqrt(2) (cos t, sin t) with t = (2a-9) pi/4 for a = 5..8."""
    out = [(0, 0)]
    for a in range(1, 5):
        t = (a - 1) * math.pi / 2
        out.append((round(math.cos(t)), round(math.sin(t))))
    for a in range(5, 9):
        t = (2 * a - 9) * math.pi / 4
        out.append((round(math.sqrt(2) * math.cos(t)), round(math.sqrt(2) * math.sin(t))))
    return out


E = velocities()
W = [Fr(4, 9)] + [Fr(1, 9)] * 4 + [Fr(1, 36)] * 4
OPP = [next(b for b in range(9) if E[b] == (-E[a][0], -E[a][1])) for a in range(9)]


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1]


def equilibrium(rho, u) -> List[Fr]:
    """eq. (feq)."""
    uu = dot(u, u)
    return [rho * W[a] * (1 + dot(E[a], u) / CS2 + (dot(E[a], u) ** 2 - CS2 * uu) / (2 * CS2 * CS2))
            for a in range(9)]


def guo_force(u, F) -> List[Fr]:
    """eq. (external-force-term) without the (1 - 1/(2 lambda)) factor."""
    out = []
    for a in range(9):
        e = E[a]
        eu = dot(e, u)
        vec = ((e[0] - u[0]) / CS2 + eu * e[0] / (CS2 * CS2),
               (e[1] - u[1]) / CS2 + eu * e[1] / (CS2 * CS2))
        out.append(W[a] * dot(vec, F))
    return out


def sym(x, a):
    return (x[a] + x[OPP[a]]) / 2


def anti(x, a):
    return (x[a] - x[OPP[a]]) / 2


def collide(f, rho_u_star_extra, tau_s, tau_a, eta, chi, uo, fb):
    """Steps (4)-(6) of the algorithm at one node, exactly."""
    rho = sum(f)
    j = (sum(E[a][0] * f[a] for a in range(9)), sum(E[a][1] * f[a] for a in range(9)))
    us = ((j[0] + fb[0] / 2) / rho, (j[1] + fb[1] / 2) / rho)
    c = Fr(1) if chi else Fr(0)
    du = tuple(c * (uo[k] - us[k]) / (2 * eta + c) for k in range(2))            # eq. (d-V)
    fvp = tuple(2 * rho * c * (uo[k] - us[k]) / (2 * eta + c) for k in range(2))  # eq. (force-density)
    u = (us[0] + du[0], us[1] + du[1])                                            # eq. (velocity-r)
    F = (fb[0] + fvp[0], fb[1] + fvp[1])
    fe = equilibrium(rho, u)
    Fa = guo_force(u, F)
    g = []
    for a in range(9):
        omega = -(sym(f, a) - sym(fe, a)) / tau_s - (anti(f, a) - anti(fe, a)) / tau_a
        g.append(f[a] + omega + (1 - 1 / (2 * tau_s)) * sym(Fa, a) + (1 - 1 / (2 * tau_a)) * anti(Fa, a))
    return g, (rho, u[0], u[1], fvp[0], fvp[1])


def run(nx: int, ny: int, tau_plus, magic_lambda, eta, bc: Sequence[str], rho_in, u_in,
        body_id, bodies, rho0_field, ux0, uy0, steps: int, fb=(Fr(0), Fr(0))):
    """Evolve exactly. ``body_id[j][i]`` ints, ``bodies`` rows (cx, cy, vx, vy,
    omega) as Fractions; initial fields as nested lists of Fractions. Returns
    (g, fields, forces) after ``steps`` steps; g[a][j][i]."""
    tau_s = Fr(tau_plus)
    tau_a = Fr(1, 2) + Fr(magic_lambda) / (tau_s - Fr(1, 2))
    eta = Fr(eta)
    g = [[[None] * nx for _ in range(ny)] for _ in range(9)]
    for j in range(ny):
        for i in range(nx):
            fe = equilibrium(rho0_field[j][i], (ux0[j][i], uy0[j][i]))
            for a in range(9):
                g[a][j][i] = fe[a]
    inflow = equilibrium(Fr(rho_in), (Fr(u_in[0]), Fr(u_in[1])))
    west, east = bc[0], bc[1]
    fields = None
    forces = []
    for _ in range(steps):
        new = [[[None] * nx for _ in range(ny)] for _ in range(9)]
        fields = [[[None] * nx for _ in range(ny)] for _ in range(5)]
        fsum: Dict[int, List[Fr]] = {}
        for j in range(ny):
            for i in range(nx):
                f = []
                for a in range(9):
                    si, sj = i - E[a][0], (j - E[a][1]) % ny
                    if 0 <= si < nx:
                        f.append(g[a][sj][si])
                        continue
                    side = west if si < 0 else east
                    if side == "periodic":
                        f.append(g[a][sj][si % nx])
                    elif side == "inflow_eq":
                        f.append(inflow[a])
                    else:
                        f.append(g[a][sj][0 if si < 0 else nx - 1])
                b = body_id[j][i]
                if b > 0:
                    cx, cy, vx, vy, om = bodies[b - 1]
                    uo = (vx - om * (j - cy), vy + om * (i - cx))
                else:
                    uo = (Fr(0), Fr(0))
                gout, fl = collide(f, None, tau_s, tau_a, eta, b > 0, uo, fb)
                for a in range(9):
                    new[a][j][i] = gout[a]
                for q in range(5):
                    fields[q][j][i] = fl[q]
                if b > 0:
                    acc = fsum.setdefault(b, [Fr(0), Fr(0)])
                    acc[0] -= fl[3]
                    acc[1] -= fl[4]
        g = new
        forces.append(fsum)
    return g, fields, forces
