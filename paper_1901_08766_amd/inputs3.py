"""Seeded synthetic inputs for the three-dimensional (D3Q19) TRT-LBM-VP solver.

Like ``inputs`` (the 2-D generators), this module is shared by the FP64 oracle
and the HIP library and holds no part of the method's arithmetic: it describes
problems (grids, masks, body tables, sides, initial fields).

Conventions: node (i, j, k) sits at x = i, y = j, z = k; host arrays are
[k][j][i] with x fastest. The mask is binary and node-centred (a node is solid
when its centre lies in the closed body, evaluated in FP64); ``body_id`` is 0
for fluid and b for the b-th body. Each body moves rigidly,
U_O(x) = V + omega x (x - c), given as the row (cx, cy, cz, vx, vy, vz, wx, wy, wz).
The x sides are periodic, equilibrium inflow or zero-gradient outflow; the y and
z sides are periodic. All randomness is numpy ``Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

from .inputs import INFLOW_EQ, OUTFLOW, PERIODIC, Problem, tau_plus_from_viscosity, viscosity_from_re

BODY_COLS = 9
SPHERE_SHAPE = (512, 256, 256)   # nx, ny, nz of the sphere workload


@dataclasses.dataclass
class Problem3:
    name: str
    nx: int
    ny: int
    nz: int
    tau_plus: float
    magic_lambda: float
    eta: float
    rho0: float = 1.0
    bc: Tuple[str, str] = (PERIODIC, PERIODIC)      # west, east (y and z are periodic)
    rho_in: float = 1.0
    u_in: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    mask: Optional[np.ndarray] = None                # uint8 [nz, ny, nx]
    bodies: Optional[np.ndarray] = None              # float64 [n_bodies, 9]
    rho_init: Optional[np.ndarray] = None            # float64 [nz, ny, nx] or None (= rho0)
    ux_init: Optional[np.ndarray] = None
    uy_init: Optional[np.ndarray] = None
    uz_init: Optional[np.ndarray] = None
    steps: int = 0
    u_ref: float = 0.0
    l_ref: float = 1.0

    @property
    def n_bodies(self) -> int:
        return 0 if self.bodies is None else int(self.bodies.shape[0])

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def mask_or_empty(self) -> np.ndarray:
        if self.mask is None:
            return np.zeros((self.nz, self.ny, self.nx), dtype=np.uint8)
        return self.mask

    def bodies_or_empty(self) -> np.ndarray:
        if self.bodies is None:
            return np.zeros((0, BODY_COLS), dtype=np.float64)
        return self.bodies


def _grid(nx: int, ny: int, nz: int):
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    return x, y, z


def paint_sphere(mask: np.ndarray, cx: float, cy: float, cz: float, r: float, body_id: int) -> None:
    nz, ny, nx = mask.shape
    x, y, z = _grid(nx, ny, nz)
    inside = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
    mask[inside] = body_id


def _paint_sphere_window(mask: np.ndarray, cx: float, cy: float, cz: float, r: float, body_id: int) -> None:
    """paint_sphere evaluated on the sphere's bounding box only (large grids)."""
    nz, ny, nx = mask.shape
    lo = [max(0, int(math.floor(c - r)) - 1) for c in (cx, cy, cz)]
    hi = [min(n, int(math.ceil(c + r)) + 2) for c, n in ((cx, nx), (cy, ny), (cz, nz))]
    x = np.arange(lo[0], hi[0], dtype=np.float64)[None, None, :]
    y = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None]
    z = np.arange(lo[2], hi[2], dtype=np.float64)[:, None, None]
    win = mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    win[(x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r] = body_id


def huge_domain3(nx: int = 1024, ny: int = 1024, nz: int = 640, seed: int = 9, n_spheres: int = 4,
                 u: float = 0.05, tau_plus: float = 0.6) -> Problem3:
    """A 3-D domain past 32-bit element offsets: 1024 x 1024 x 640 nodes, 1.27e10
    populations per lattice. Spheres turning about random axes and translating,
    half of them in the last planes; a uniform body force drives every node from
    rest (no host field arrays), inflow and zero-gradient outflow x sides."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    rows = []
    for k in range(n_spheres):
        r = float(rng.uniform(5.0, 24.0))
        far = k % 2 == 1
        c = [float(rng.uniform(n - 200, n - 40) if far else rng.uniform(40, n - 40)) for n in (nx, ny, nz)]
        _paint_sphere_window(mask, c[0], c[1], c[2], r, k + 1)
        v = [float(rng.uniform(-0.3, 0.3)) * u for _ in range(3)]
        om = [float(rng.uniform(-1, 1)) * u / r for _ in range(3)]
        rows.append(c + v + om)
    return Problem3(name=f"huge{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, tau_plus=tau_plus, magic_lambda=0.25,
                    eta=1e-4, bc=(INFLOW_EQ, OUTFLOW), rho_in=1.0, u_in=(u, 0.0, 0.0),
                    body_force=(2e-5, -1e-5, 5e-6), mask=mask, bodies=np.array(rows), u_ref=u, l_ref=1.0)


def paint_box(mask: np.ndarray, lo: Tuple[int, int, int], hi: Tuple[int, int, int], body_id: int) -> None:
    """Nodes lo <= (i, j, k) < hi, given as (x, y, z) bounds."""
    mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = body_id


def extrude(p: Problem, nz: int) -> Problem3:
    """The z-invariant 3-D problem of a 2-D one: every z plane holds the 2-D mask
    and fields, u_z = 0, and each body turns about the z axis (its row
    (cx, cy, vx, vy, omega) becomes (cx, cy, 0, vx, vy, 0, 0, 0, omega))."""
    def rep(a):
        return None if a is None else np.ascontiguousarray(np.broadcast_to(a, (nz,) + a.shape))

    b2 = p.bodies_or_empty()
    b3 = np.zeros((b2.shape[0], BODY_COLS))
    b3[:, 0], b3[:, 1], b3[:, 3], b3[:, 4], b3[:, 8] = b2[:, 0], b2[:, 1], b2[:, 2], b2[:, 3], b2[:, 4]
    bc = (p.bc[0], p.bc[1])
    if p.bc[2] != PERIODIC or p.bc[3] != PERIODIC:
        raise ValueError("only problems with periodic y sides extrude")
    return Problem3(name=f"{p.name}_z{nz}", nx=p.nx, ny=p.ny, nz=nz, tau_plus=p.tau_plus,
                    magic_lambda=p.magic_lambda, eta=p.eta, rho0=p.rho0, bc=bc, rho_in=p.rho_in,
                    u_in=(p.u_in[0], p.u_in[1], 0.0), body_force=(p.body_force[0], p.body_force[1], 0.0),
                    mask=rep(p.mask_or_empty()), bodies=b3 if b2.shape[0] else None,
                    rho_init=rep(p.rho_init), ux_init=rep(p.ux_init), uy_init=rep(p.uy_init),
                    uz_init=None if p.ux_init is None else np.zeros((nz, p.ny, p.nx)),
                    steps=p.steps, u_ref=p.u_ref, l_ref=p.l_ref)


def permute_axes(p: Problem3, order: Tuple[int, int, int]) -> Problem3:
    """Relabel the axes of a fully periodic problem: new axis d is old axis
    order[d] (0 = x, 1 = y, 2 = z). Arrays, body rows and vectors follow."""
    if p.bc != (PERIODIC, PERIODIC):
        raise ValueError("axis relabelling needs periodic x sides")
    old_n = (p.nx, p.ny, p.nz)
    n = tuple(old_n[order[d]] for d in range(3))
    # array axes are (z, y, x) = (2, 1, 0): new array axis for new dim d holds old dim order[d]
    perm = tuple(2 - order[2 - a] for a in range(3))

    def arr(a):
        return None if a is None else np.ascontiguousarray(np.transpose(a, perm))

    def vec(v):
        return tuple(v[order[d]] for d in range(3))

    vels = [p.ux_init, p.uy_init, p.uz_init]
    b = p.bodies_or_empty()
    nb = np.zeros_like(b)
    even = order in ((0, 1, 2), (1, 2, 0), (2, 0, 1))
    for d in range(3):
        nb[:, d] = b[:, order[d]]
        nb[:, 3 + d] = b[:, 3 + order[d]]
        # omega is a pseudo-vector: an odd relabelling of the axes flips it
        nb[:, 6 + d] = b[:, 6 + order[d]] * (1.0 if even else -1.0)
    return Problem3(name=f"{p.name}_perm{''.join(map(str, order))}", nx=n[0], ny=n[1], nz=n[2],
                    tau_plus=p.tau_plus, magic_lambda=p.magic_lambda, eta=p.eta, rho0=p.rho0, bc=p.bc,
                    rho_in=p.rho_in, u_in=vec(p.u_in), body_force=vec(p.body_force), mask=arr(p.mask),
                    bodies=nb if b.shape[0] else None, rho_init=arr(p.rho_init),
                    ux_init=arr(vels[order[0]]), uy_init=arr(vels[order[1]]), uz_init=arr(vels[order[2]]),
                    steps=p.steps, u_ref=p.u_ref, l_ref=p.l_ref)


def random_state_problem3(nx: int, ny: int, nz: int, seed, n_spheres: int = 3,
                          bc=(INFLOW_EQ, OUTFLOW), tau_plus: float = 0.7, magic_lambda: float = 0.25,
                          eta: float = 1e-4, u: float = 0.05, moving: bool = True,
                          body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)) -> Problem3:
    """A small random problem for parity tests: random spheres (translating and
    turning about random axes), random initial fields of moderate amplitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    rows = []
    for b in range(n_spheres):
        r = float(rng.uniform(1.0, max(1.5, min(nx, ny, nz) / 5.0)))
        c = [float(rng.uniform(0, n)) for n in (nx, ny, nz)]
        paint_sphere(mask, c[0], c[1], c[2], r, b + 1)
        v = rng.uniform(-1, 1, size=3) * u * 0.3 if moving else np.zeros(3)
        w = rng.uniform(-1, 1, size=3) * u / r if moving else np.zeros(3)
        rows.append(c + list(v) + list(w))
    bodies = np.array(rows) if rows else None
    shape = (nz, ny, nx)
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, size=shape)
    ux = u + 0.3 * u * rng.uniform(-1, 1, size=shape)
    uy = 0.3 * u * rng.uniform(-1, 1, size=shape)
    uz = 0.3 * u * rng.uniform(-1, 1, size=shape)
    return Problem3(name=f"random{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, tau_plus=tau_plus,
                    magic_lambda=magic_lambda, eta=eta, bc=tuple(bc), rho_in=1.0, u_in=(u, 0.0, 0.0),
                    body_force=body_force, mask=mask, bodies=bodies, rho_init=rho, ux_init=ux, uy_init=uy,
                    uz_init=uz, u_ref=u, l_ref=1.0)


def sphere(nx: int = SPHERE_SHAPE[0], ny: int = SPHERE_SHAPE[1], nz: int = SPHERE_SHAPE[2], d: float = 32.0,
           cx: Optional[float] = None,
           u: float = 0.05, re: float = 300.0, magic_lambda: float = 0.25, eta: float = 1e-4,
           amp: float = 0.01, seed: int = 11, steps: int = 0) -> Problem3:
    """Uniform flow past a fixed sphere (the 3-D counterpart of the cylinder
    case): equilibrium inflow at (u, 0, 0) on the west side, zero-gradient
    outflow on the east, periodic y and z, Re = u d / nu. The initial field is
    the free stream with a small seeded transverse perturbation to break the
    symmetry of the wake."""
    cx = nx / 4.0 if cx is None else cx
    cy, cz = ny / 2.0, nz / 2.0
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    paint_sphere(mask, cx, cy, cz, d / 2.0, 1)
    bodies = np.array([[cx, cy, cz, 0, 0, 0, 0, 0, 0]], dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    fluid = mask == 0
    ux = np.where(fluid, u, 0.0)
    uy = np.where(fluid, amp * u * rng.uniform(-1, 1, size=shape).astype(np.float64), 0.0)
    uz = np.where(fluid, amp * u * rng.uniform(-1, 1, size=shape).astype(np.float64), 0.0)
    tau = tau_plus_from_viscosity(viscosity_from_re(u, d, re))
    return Problem3(name=f"sphere{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, tau_plus=tau,
                    magic_lambda=magic_lambda, eta=eta, bc=(INFLOW_EQ, OUTFLOW), rho_in=1.0,
                    u_in=(u, 0.0, 0.0), mask=mask, bodies=bodies, ux_init=ux, uy_init=uy, uz_init=uz,
                    steps=steps, u_ref=u, l_ref=d)


ENSEMBLE3_NX = (96, 128, 160)
ENSEMBLE3_NYZ = (32, 48, 64)


def ensemble3(n: int = 64, seed: int = 5) -> List[Problem3]:
    """An ensemble of independent sphere domains of uneven sizes (the 3-D
    counterpart of the channel ensemble): nx from ENSEMBLE3_NX, ny and nz from
    ENSEMBLE3_NYZ, sphere diameter ~ U[8, min(ny, nz) / 3] at a random height,
    Re ~ U[20, 50] (tau+ >= 0.524), each with its own seeded perturbation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        nx = int(ENSEMBLE3_NX[int(rng.integers(len(ENSEMBLE3_NX)))])
        ny, nz = (int(ENSEMBLE3_NYZ[int(rng.integers(len(ENSEMBLE3_NYZ)))]) for _ in range(2))
        d = float(rng.uniform(8.0, min(ny, nz) / 3.0))
        re = float(rng.uniform(20.0, 50.0))
        p = sphere(nx, ny, nz, d=d, re=re, seed=int(rng.integers(1 << 31)))
        out.append(dataclasses.replace(p, name=f"ens3_{k}_{p.name}"))
    return out


def shear_wave(n: int = 32, u0: float = 1e-3, axis_u: int = 0, axis_k: int = 2, tau_plus: float = 0.8,
               magic_lambda: float = 0.25, m: int = 1) -> Problem3:
    """A decaying shear wave on an n^3 periodic box: velocity component axis_u
    equal to u0 sin(2 pi m s / n) along axis_k, everything else at rest."""
    if axis_u == axis_k:
        raise ValueError("a shear wave needs distinct velocity and wave axes")
    x, y, z = _grid(n, n, n)
    s = (x, y, z)[axis_k]
    prof = np.broadcast_to(u0 * np.sin(2.0 * math.pi * m * s / n), (n, n, n)).copy()
    vel = [np.zeros((n, n, n)) for _ in range(3)]
    vel[axis_u] = prof
    return Problem3(name=f"shear{n}_{axis_u}{axis_k}", nx=n, ny=n, nz=n, tau_plus=tau_plus,
                    magic_lambda=magic_lambda, eta=1e-4, ux_init=vel[0], uy_init=vel[1], uz_init=vel[2],
                    u_ref=u0, l_ref=float(n))


def plate_channel(nz: int = 24, nxy: int = 4, wall: int = 2, fx: float = 1e-6, tau_plus: float = 0.9,
                  magic_lambda: float = 0.25, eta: float = 1e-4) -> Problem3:
    """Body-force driven flow between two plates normal to z (``wall`` solid
    planes at the bottom and at the top, one fixed body), periodic elsewhere."""
    mask = np.zeros((nz, nxy, nxy), dtype=np.uint8)
    mask[:wall] = 1
    mask[nz - wall:] = 1
    bodies = np.array([[nxy / 2.0, nxy / 2.0, nz / 2.0, 0, 0, 0, 0, 0, 0]], dtype=np.float64)
    return Problem3(name=f"plates{nz}", nx=nxy, ny=nxy, nz=nz, tau_plus=tau_plus, magic_lambda=magic_lambda,
                    eta=eta, body_force=(fx, 0.0, 0.0), mask=mask, bodies=bodies)


def slab(p: Problem3, k0: int, n: int) -> Problem3:
    """Planes k0 .. k0 + n - 1 (taken modulo nz) of a problem as a problem of their
    own, periodic along z over the n planes, with each body centre moved to slab
    coordinates at its image nearest the slab. A node update in the middle plane
    of a 3-plane slab reads that slab only. The initial fields are cut the same
    way."""
    ks = [(k0 + s) % p.nz for s in range(n)]

    def cut(a):
        return None if a is None else np.ascontiguousarray(a[ks])

    b = p.bodies_or_empty().copy()
    rel = b[:, 2] - k0                                  # the centre's image nearest the slab
    b[:, 2] = rel - p.nz * np.round((rel - 0.5 * (n - 1)) / p.nz)
    return Problem3(name=f"{p.name}_slab{k0}+{n}", nx=p.nx, ny=p.ny, nz=n, tau_plus=p.tau_plus,
                    magic_lambda=p.magic_lambda, eta=p.eta, rho0=p.rho0, bc=p.bc, rho_in=p.rho_in, u_in=p.u_in,
                    body_force=p.body_force, mask=cut(p.mask_or_empty()), bodies=b if b.shape[0] else None,
                    rho_init=cut(p.rho_init), ux_init=cut(p.ux_init), uy_init=cut(p.uy_init),
                    uz_init=cut(p.uz_init), steps=p.steps, u_ref=p.u_ref, l_ref=p.l_ref)
