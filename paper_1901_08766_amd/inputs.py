"""Seeded synthetic inputs for the TRT-LBM-VP solver: grids, masks, body tables,
boundary sides and initial fields.

This module is the only code shared by the FP64 oracle and the HIP library. It
holds no part of the method's arithmetic (no equilibrium, collision, forcing or
penalization): it describes problems. Both sides receive the very same host
arrays from it.

Geometry conventions (paper Sec. 2.2, eq. mask function): node (i, j) sits at
x = i, y = j; host arrays are row-major [j][i] with x fastest. The mask is
binary and node-centred: a node is solid when its centre lies inside the closed
body (ties count as solid), evaluated in FP64. ``body_id`` is 0 for fluid and k
for the k-th body (1-based); chi = (body_id > 0).

Each body moves rigidly: U_O(x) = (vx, vy) + omega * z_hat x (x - c)
(paper Sec. 2.2, eq. boundary-condition; the paper's experiments rotate bodies
in Secs. 3.1 and 3.4). A body is the row (cx, cy, vx, vy, omega).

All randomness is numpy ``Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PERIODIC = "periodic"
INFLOW_EQ = "inflow_eq"
OUTFLOW = "outflow_zero_grad"


@dataclasses.dataclass
class Problem:
    """One solve: everything the paper's problem statement fixes (Sec. 2)."""

    name: str
    nx: int
    ny: int
    tau_plus: float
    magic_lambda: float
    eta: float
    rho0: float = 1.0
    bc: Tuple[str, str, str, str] = (PERIODIC, PERIODIC, PERIODIC, PERIODIC)  # west, east, south, north
    rho_in: float = 1.0
    u_in: Tuple[float, float] = (0.0, 0.0)
    body_force: Tuple[float, float] = (0.0, 0.0)
    mask: Optional[np.ndarray] = None        # uint8 [ny, nx]
    bodies: Optional[np.ndarray] = None      # float64 [n_bodies, 5]
    rho_init: Optional[np.ndarray] = None    # float64 [ny, nx] or None (= rho0)
    ux_init: Optional[np.ndarray] = None     # float64 [ny, nx] or None (= 0)
    uy_init: Optional[np.ndarray] = None
    steps: int = 0
    u_ref: float = 0.0                       # U_inf for force coefficients
    l_ref: float = 1.0                       # D (or chord) for force coefficients
    moving: bool = False                     # bodies move rigidly (the mask follows them)

    @property
    def n_bodies(self) -> int:
        return 0 if self.bodies is None else int(self.bodies.shape[0])

    def mask_or_empty(self) -> np.ndarray:
        if self.mask is None:
            return np.zeros((self.ny, self.nx), dtype=np.uint8)
        return self.mask

    def bodies_or_empty(self) -> np.ndarray:
        if self.bodies is None:
            return np.zeros((0, 5), dtype=np.float64)
        return self.bodies


# ----------------------------------------------------------------------------
# parameters from physical numbers
# ----------------------------------------------------------------------------

def viscosity_from_re(u: float, length: float, re: float) -> float:
    """Re = U L / nu (paper Sec. 3, definition of Re)."""
    return u * length / re


def tau_plus_from_viscosity(nu: float) -> float:
    """Symmetric relaxation time from the kinematic viscosity in lattice units.

    The paper prints tau_s = nu / (c_s^2 dt) (Sec. 2.1, below eq. feq); with the
    magic-parameter relation (tau_s - 1/2)(tau_a - 1/2) this only makes sense for
    the standard lattice relation nu = c_s^2 (tau_s - 1/2), which is used here.
    """
    return 3.0 * nu + 0.5


# ----------------------------------------------------------------------------
# geometry rasterizers (FP64, node-centred, ties solid)
# ----------------------------------------------------------------------------

def _grid(nx: int, ny: int):
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    return x, y


def paint_disk(mask: np.ndarray, cx: float, cy: float, r: float, body_id: int) -> None:
    """Mark nodes with (x-cx)^2 + (y-cy)^2 <= r^2 as ``body_id``."""
    ny, nx = mask.shape
    x, y = _grid(nx, ny)
    inside = (x - cx) ** 2 + (y - cy) ** 2 <= r * r
    mask[inside] = body_id


def paint_outside_disk(mask: np.ndarray, cx: float, cy: float, r: float, body_id: int) -> None:
    """Mark nodes with (x-cx)^2 + (y-cy)^2 >= r^2 as ``body_id``."""
    ny, nx = mask.shape
    x, y = _grid(nx, ny)
    outside = (x - cx) ** 2 + (y - cy) ** 2 >= r * r
    mask[outside] = body_id


def naca4_half_thickness(xi: np.ndarray, chord: float, t: float = 0.12) -> np.ndarray:
    """Half thickness of a symmetric NACA 4-digit section at chordwise distance xi
    from the leading edge (public closed form, closed trailing edge)."""
    s = np.clip(xi / chord, 0.0, 1.0)
    return 5.0 * t * chord * (0.2969 * np.sqrt(s) - 0.1260 * s - 0.3516 * s ** 2
                              + 0.2843 * s ** 3 - 0.1036 * s ** 4)


def paint_naca0012(mask: np.ndarray, le_x: float, le_y: float, chord: float,
                   aoa_deg: float, pivot: Tuple[float, float], body_id: int) -> None:
    """NACA-0012 whose unrotated chord runs from (le_x, le_y) in +x, then rotated
    nose-up by ``aoa_deg`` about ``pivot`` (flow in +x, y up)."""
    ny, nx = mask.shape
    x, y = _grid(nx, ny)
    a = math.radians(aoa_deg)
    px, py = pivot
    dx, dy = x - px, y - py
    # undo the nose-up (clockwise) rotation: rotate the node by +a about the pivot
    xr = dx * math.cos(a) - dy * math.sin(a) + px
    yr = dx * math.sin(a) + dy * math.cos(a) + py
    xi = xr - le_x
    inside = (xi >= 0.0) & (xi <= chord) & (np.abs(yr - le_y) <= naca4_half_thickness(xi, chord))
    mask[inside] = body_id


def body_velocity(bodies: np.ndarray, mask: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Rigid-body velocity of each solid node (0 in the fluid), FP64. Used only to
    set initial fields of solid nodes to their body's velocity."""
    ny, nx = mask.shape
    x, y = _grid(nx, ny)
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    for k in range(bodies.shape[0]):
        cx, cy, vx, vy, om = bodies[k]
        sel = mask == (k + 1)
        ux_k = vx - om * (y - cy)
        uy_k = vy + om * (x - cx)
        ux[sel] = np.broadcast_to(ux_k, (ny, nx))[sel]
        uy[sel] = np.broadcast_to(uy_k, (ny, nx))[sel]
    return ux, uy


def seeded_inflow_init(mask: np.ndarray, bodies: np.ndarray, u: float, amp: float,
                       seed) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """rho = 1, u = (U, amp*U*xi) with xi ~ U[-1, 1] iid per fluid node; solid
    nodes take their body velocity. ``amp`` = 0 gives the noise-free field."""
    ny, nx = mask.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.uniform(-1.0, 1.0, size=(ny, nx))
    rho = np.ones((ny, nx))
    ux = np.full((ny, nx), u)
    uy = amp * u * xi
    bux, buy = body_velocity(bodies, mask)
    solid = mask > 0
    ux[solid] = bux[solid]
    uy[solid] = buy[solid]
    return rho, ux, uy


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def couette(n: int = 64, r_in: float = 12.0, r_out: float = 28.0, u0: float = 0.01,
            tau_plus: float = 0.8, magic_lambda: float = 0.25, eta: float = 1e-4,
            steps: int = 2000) -> Problem:
    """Cylindrical Couette flow (paper Sec. 3.1) on an n x n fully periodic grid.

    Centre ((n-1)/2, (n-1)/2); solid r <= r_in rotates counter-clockwise with
    surface speed u0 (omega = u0 / r_in); solid r >= r_out is fixed. Fluid at
    rest with rho = 1. The defaults are the 64 x 64 case.
    """
    c = (n - 1) / 2.0
    mask = np.zeros((n, n), dtype=np.uint8)
    paint_outside_disk(mask, c, c, r_out, 2)
    paint_disk(mask, c, c, r_in, 1)
    bodies = np.array([[c, c, 0.0, 0.0, u0 / r_in],
                       [c, c, 0.0, 0.0, 0.0]])
    return Problem(name=f"couette{n}", nx=n, ny=n, tau_plus=tau_plus, magic_lambda=magic_lambda,
                   eta=eta, mask=mask, bodies=bodies, steps=steps, u_ref=u0, l_ref=2 * r_in)


def cylinder(nx: int = 1024, ny: int = 512, d: float = 40.0, cx: float = 256.0, cy: float = 256.0,
             u: float = 0.05, re: float = 100.0, magic_lambda: float = 3.0 / 16.0,
             eta: float = 1e-4, noise: bool = True, seed=2, steps: int = 200_000) -> Problem:
    """Single fixed circular cylinder in a channel (paper Sec. 3.2): equilibrium
    inflow U on the west, zero-gradient outflow on the east, periodic north and
    south. Defaults: 1024 x 512, D = 40 at (256, 256), Re = 100."""
    mask = np.zeros((ny, nx), dtype=np.uint8)
    paint_disk(mask, cx, cy, d / 2.0, 1)
    bodies = np.array([[cx, cy, 0.0, 0.0, 0.0]])
    rho, ux, uy = seeded_inflow_init(mask, bodies, u, 1e-3 if noise else 0.0, seed)
    nu = viscosity_from_re(u, d, re)
    return Problem(name=f"cylinder{nx}x{ny}_re{re:g}", nx=nx, ny=ny,
                   tau_plus=tau_plus_from_viscosity(nu), magic_lambda=magic_lambda, eta=eta,
                   bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC), rho_in=1.0, u_in=(u, 0.0),
                   mask=mask, bodies=bodies, rho_init=rho, ux_init=ux, uy_init=uy,
                   steps=steps, u_ref=u, l_ref=d)


def large_domain(scale: int = 1, u: float = 0.04, re: float = 200.0, magic_lambda: float = 0.25,
                 eta: float = 1e-4, seed=3, noise: bool = True, steps: Optional[int] = None,
                 moving: bool = False) -> Problem:
    """Large single domain (8192 x 4096 at scale 1) holding two counter-rotating
    cylinders (Sec. 3.4), a tandem pair (Sec. 3.3.1) and a NACA-0012 airfoil
    (Sec. 3.5). All lengths are divided by ``scale``; U and Re are kept.

    Bodies (1-based ids): 1 upper rotating (clockwise), 2 lower rotating
    (counter-clockwise), surface speed U, gap-side surfaces moving upstream;
    3 tandem upstream, 4 tandem downstream (centre spacing 2D); 5 the airfoil,
    chord 5D, 5 degrees nose-up about its quarter chord.

    ``moving``: the mask follows the bodies (a time-dependent chi): the upstream
    tandem cylinder crosses the stream at 0.1 U and the airfoil keeps pitching
    nose-up (clockwise) about its quarter chord, its trailing edge at 0.3 U; the rotating
    cylinders turn their masks with their surfaces.
    """
    s = float(scale)
    nx, ny = 8192 // scale, 4096 // scale
    d = 160.0 / s
    r = d / 2.0
    om = 2.0 * u / d
    mask = np.zeros((ny, nx), dtype=np.uint8)
    rot_x, rot_y, half_gap = 1280.0 / s, 3200.0 / s, 120.0 / s
    tan_y, tan_x0, tan_x1 = 900.0 / s, 1280.0 / s, 1600.0 / s
    chord, le_x, le_y = 800.0 / s, 1000.0 / s, 2048.0 / s
    pivot = (le_x + chord / 4.0, le_y)
    paint_disk(mask, rot_x, rot_y + half_gap, r, 1)
    paint_disk(mask, rot_x, rot_y - half_gap, r, 2)
    paint_disk(mask, tan_x0, tan_y, r, 3)
    paint_disk(mask, tan_x1, tan_y, r, 4)
    paint_naca0012(mask, le_x, le_y, chord, 5.0, pivot, 5)
    bodies = np.array([
        [rot_x, rot_y + half_gap, 0.0, 0.0, -om],
        [rot_x, rot_y - half_gap, 0.0, 0.0, +om],
        [tan_x0, tan_y, 0.0, 0.0, 0.0],
        [tan_x1, tan_y, 0.0, 0.0, 0.0],
        [pivot[0], pivot[1], 0.0, 0.0, 0.0],
    ])
    if moving:
        bodies[2, 3] = 0.1 * u
        bodies[4, 4] = -0.3 * u / (0.75 * chord)
    rho, ux, uy = seeded_inflow_init(mask, bodies, u, 1e-3 if noise else 0.0, seed)
    nu = viscosity_from_re(u, d, re)
    if steps is None:
        steps = 50_000 // scale
    return Problem(name=f"large{nx}x{ny}" + ("-moving" if moving else ""), nx=nx, ny=ny,
                   tau_plus=tau_plus_from_viscosity(nu),
                   magic_lambda=magic_lambda, eta=eta, bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC),
                   rho_in=1.0, u_in=(u, 0.0), mask=mask, bodies=bodies, rho_init=rho,
                   ux_init=ux, uy_init=uy, steps=steps, u_ref=u, l_ref=d, moving=moving)


ENSEMBLE_SIZES = ((128, 128), (256, 128), (512, 256), (1024, 512))


def ensemble_domain(rng: np.random.Generator, d_index: int, seed: int = 4, u: float = 0.05,
                    magic_lambda: float = 0.25, eta: float = 1e-4, steps: int = 20_000,
                    sizes: Sequence[Tuple[int, int]] = ENSEMBLE_SIZES) -> Problem:
    """One random multi-cylinder channel domain drawn from ``rng``: size from
    ``sizes``, 1-4 non-overlapping cylinders (integer radius 8..min(40, ny/4),
    surface gap >= 4, rejection with at most 100 tries each), Re ~ U[40, 200] on
    the largest diameter; channel boundaries as for a single cylinder."""
    nx, ny = sizes[int(rng.integers(len(sizes)))]
    n_cyl = int(rng.integers(1, 5))
    r_hi = min(40, ny // 4)
    placed: List[Tuple[float, float, float]] = []
    for _ in range(n_cyl):
        r = float(rng.integers(8, r_hi + 1))
        for _try in range(100):
            cx = float(rng.uniform(r + nx / 8.0, nx / 2.0))
            cy = float(rng.uniform(r + 4.0, ny - r - 4.0))
            ok = all(math.hypot(cx - px, cy - py) >= r + pr + 4.0 for px, py, pr in placed)
            if ok:
                placed.append((cx, cy, r))
                break
    mask = np.zeros((ny, nx), dtype=np.uint8)
    for k, (cx, cy, r) in enumerate(placed):
        paint_disk(mask, cx, cy, r, k + 1)
    bodies = np.array([[cx, cy, 0.0, 0.0, 0.0] for cx, cy, _ in placed])
    d_ref = 2.0 * max(r for _, _, r in placed)
    re = float(rng.uniform(40.0, 200.0))
    nu = viscosity_from_re(u, d_ref, re)
    rho, ux, uy = seeded_inflow_init(mask, bodies, u, 1e-3, (seed, d_index))
    return Problem(name=f"ens{d_index}_{nx}x{ny}", nx=nx, ny=ny, tau_plus=tau_plus_from_viscosity(nu),
                   magic_lambda=magic_lambda, eta=eta, bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC),
                   rho_in=1.0, u_in=(u, 0.0), mask=mask, bodies=bodies, rho_init=rho,
                   ux_init=ux, uy_init=uy, steps=steps, u_ref=u, l_ref=d_ref)


def ensemble(n: int = 256, seed: int = 4, **kw) -> List[Problem]:
    """The batched ensemble: ``n`` independent random channel domains."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [ensemble_domain(rng, d, seed=seed, **kw) for d in range(n)]


def airfoil_request(rng: np.random.Generator, r_index: int, seed: int, u: float = 0.05,
                    sizes: Sequence[Tuple[int, int]] = ENSEMBLE_SIZES) -> Problem:
    """A NACA-0012 channel domain: chord ny/2, quarter chord at (0.3 nx, ny/2),
    nose-up attack angle ~ U[0, 10] degrees, Re on the chord ~ U[40, 200]."""
    nx, ny = sizes[int(rng.integers(len(sizes)))]
    chord = ny / 2.0
    aoa = float(rng.uniform(0.0, 10.0))
    pivot = (0.3 * nx, ny / 2.0)
    le_x = pivot[0] - chord / 4.0
    mask = np.zeros((ny, nx), dtype=np.uint8)
    paint_naca0012(mask, le_x, pivot[1], chord, aoa, pivot, 1)
    bodies = np.array([[pivot[0], pivot[1], 0.0, 0.0, 0.0]])
    re = float(rng.uniform(40.0, 200.0))
    nu = viscosity_from_re(u, chord, re)
    rho, ux, uy = seeded_inflow_init(mask, bodies, u, 1e-3, (seed, r_index))
    return Problem(name=f"foil{r_index}_{nx}x{ny}", nx=nx, ny=ny, tau_plus=tau_plus_from_viscosity(nu),
                   magic_lambda=0.25, eta=1e-4, bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC),
                   rho_in=1.0, u_in=(u, 0.0), mask=mask, bodies=bodies, rho_init=rho,
                   ux_init=ux, uy_init=uy, u_ref=u, l_ref=chord)


@dataclasses.dataclass
class Request:
    """One solve request of the serving stream."""
    rid: int
    arrival: float          # seconds from stream start
    problem: Problem


def request_stream(rate: float, n: int, seed: int = 5, step_lo: int = 1000,
                   step_hi: int = 50_000, sizes: Sequence[Tuple[int, int]] = ENSEMBLE_SIZES) -> List[Request]:
    """Poisson arrivals at ``rate`` req/s; each request is an ensemble-style
    cylinder domain with probability 1/2, else a NACA-0012 domain; step counts
    are log-uniform in [step_lo, step_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < 0.5:
            p = ensemble_domain(rng, k, seed=seed, sizes=sizes)
        else:
            p = airfoil_request(rng, k, seed, sizes=sizes)
        p.steps = int(round(math.exp(rng.uniform(math.log(step_lo), math.log(step_hi)))))
        out.append(Request(rid=k, arrival=t, problem=p))
    return out


def moving_bodies(nx: int = 160, ny: int = 96, seed: int = 7, bc=(PERIODIC,) * 4, u_in: float = 0.0,
                  tau_plus: float = 0.7, magic_lambda: float = 0.25, eta: float = 1e-4) -> Problem:
    """Rigidly moving bodies (time-dependent mask): a disk translating with
    V = (0.03, 0.012), an elliptic body turning at omega = 0.004 about its centre
    while drifting, and a NACA-0012 (chord 24) pitching at omega = -0.003 about
    its quarter chord. Fluid with small random velocities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    paint_disk(mask, 40.0, 30.0, 7.0, 1)
    x, y = _grid(nx, ny)
    ex, ey = 90.0, 62.0
    ang = math.radians(25.0)
    xr = (x - ex) * math.cos(ang) + (y - ey) * math.sin(ang)
    yr = -(x - ex) * math.sin(ang) + (y - ey) * math.cos(ang)
    mask[((xr / 10.0) ** 2 + (yr / 4.0) ** 2 <= 1.0) & (mask == 0)] = 2
    chord, le = 24.0, (112.0, 28.0)
    pivot = (le[0] + chord / 4.0, le[1])
    foil = np.zeros_like(mask)
    paint_naca0012(foil, le[0], le[1], chord, 8.0, pivot, 3)
    mask[(foil == 3) & (mask == 0)] = 3
    bodies = np.array([[40.0, 30.0, 0.03, 0.012, 0.0],
                       [ex, ey, -0.01, 0.005, 0.004],
                       [pivot[0], pivot[1], 0.0, 0.0, -0.003]])
    u = 0.02
    rho = 1.0 + 0.002 * rng.uniform(-1, 1, size=(ny, nx))
    ux = u_in + u * rng.uniform(-1, 1, size=(ny, nx))
    uy = u * rng.uniform(-1, 1, size=(ny, nx))
    return Problem(name=f"moving{nx}x{ny}", nx=nx, ny=ny, tau_plus=tau_plus, magic_lambda=magic_lambda, eta=eta,
                   bc=tuple(bc), rho_in=1.0, u_in=(u_in, 0.0), mask=mask, bodies=bodies, rho_init=rho,
                   ux_init=ux, uy_init=uy, u_ref=max(u_in, 0.03), l_ref=14.0, moving=True)


def taylor_green(n: int = 64, u0: float = 1e-3, tau_plus: float = 0.8, magic_lambda: float = 0.25,
                 steps: int = 1000) -> Problem:
    """Taylor-Green vortex on an n x n periodic grid, no obstacle:
    u = U0 (-cos kx sin ky, sin kx cos ky), k = 2 pi / n, and the matching
    pressure p = -rho0 U0^2/4 (cos 2kx + cos 2ky), given as rho = 1 + 3 p."""
    x, y = _grid(n, n)
    k = 2.0 * math.pi / n
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    p = -0.25 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    rho = 1.0 + 3.0 * p
    return Problem(name=f"taylor_green{n}", nx=n, ny=n, tau_plus=tau_plus, magic_lambda=magic_lambda,
                   eta=1e-4, rho_init=np.broadcast_to(rho, (n, n)).copy(),
                   ux_init=np.broadcast_to(ux, (n, n)).copy(), uy_init=np.broadcast_to(uy, (n, n)).copy(),
                   steps=steps, u_ref=u0, l_ref=float(n))


def poiseuille(ny: int = 24, nx: int = 4, wall: int = 2, fx: float = 1e-6, tau_plus: float = 0.9,
               magic_lambda: float = 0.25, eta: float = 1e-4, steps: int = 20_000) -> Problem:
    """Body-force driven channel: periodic in x and y, ``wall`` solid rows at the
    bottom and at the top (one fixed body), uniform body force (fx, 0)."""
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[:wall, :] = 1
    mask[ny - wall:, :] = 1
    bodies = np.array([[nx / 2.0, ny / 2.0, 0.0, 0.0, 0.0]])
    return Problem(name=f"poiseuille{ny}", nx=nx, ny=ny, tau_plus=tau_plus, magic_lambda=magic_lambda,
                   eta=eta, body_force=(fx, 0.0), mask=mask, bodies=bodies, steps=steps)


def random_state_problem(nx: int, ny: int, seed, n_disks: int = 3, bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC),
                         tau_plus: float = 0.7, magic_lambda: float = 0.25, eta: float = 1e-4,
                         u: float = 0.05, rotating: bool = True,
                         body_force: Tuple[float, float] = (0.0, 0.0)) -> Problem:
    """A small random problem for parity tests: random disks (some rotating and
    translating), random initial fields of moderate amplitude."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    rows = []
    for k in range(n_disks):
        r = float(rng.uniform(1.0, max(1.5, min(nx, ny) / 6.0)))
        cx = float(rng.uniform(0, nx))
        cy = float(rng.uniform(0, ny))
        paint_disk(mask, cx, cy, r, k + 1)
        om = float(rng.uniform(-1, 1)) * u / r if rotating else 0.0
        vx = float(rng.uniform(-1, 1)) * u * 0.3 if rotating else 0.0
        vy = float(rng.uniform(-1, 1)) * u * 0.3 if rotating else 0.0
        rows.append([cx, cy, vx, vy, om])
    bodies = np.array(rows) if rows else np.zeros((0, 5))
    rho = 1.0 + 0.01 * rng.uniform(-1, 1, size=(ny, nx))
    ux = u + 0.3 * u * rng.uniform(-1, 1, size=(ny, nx))
    uy = 0.3 * u * rng.uniform(-1, 1, size=(ny, nx))
    return Problem(name=f"random{nx}x{ny}", nx=nx, ny=ny, tau_plus=tau_plus, magic_lambda=magic_lambda,
                   eta=eta, bc=tuple(bc), rho_in=1.0, u_in=(u, 0.0), body_force=body_force,
                   mask=mask, bodies=bodies, rho_init=rho, ux_init=ux, uy_init=uy, u_ref=u, l_ref=1.0)


def _paint_disk_window(mask: np.ndarray, cx: float, cy: float, r: float, body_id: int) -> None:
    """paint_disk evaluated on the disk's bounding box only (large grids)."""
    ny, nx = mask.shape
    x0, x1 = max(0, int(math.floor(cx - r)) - 1), min(nx, int(math.ceil(cx + r)) + 2)
    y0, y1 = max(0, int(math.floor(cy - r)) - 1), min(ny, int(math.ceil(cy + r)) + 2)
    x = np.arange(x0, x1, dtype=np.float64)[None, :]
    y = np.arange(y0, y1, dtype=np.float64)[:, None]
    win = mask[y0:y1, x0:x1]
    win[(x - cx) ** 2 + (y - cy) ** 2 <= r * r] = body_id


def huge_domain(nx: int = 32768, ny: int = 16384, seed: int = 8, n_disks: int = 6, u: float = 0.05,
                tau_plus: float = 0.6) -> Problem:
    """A domain at the size where 32-bit element offsets no longer reach: 32768 x
    16384 nodes, 4.8e9 populations per lattice (past 2^32). Rotating and
    translating disks, half of them in the last rows and columns; a uniform body
    force drives every node from rest (no host field arrays: the fluid starts at
    rho0, u = 0), inflow and zero-gradient outflow x sides."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    rows = []
    for k in range(n_disks):
        r = float(rng.uniform(6.0, 40.0))
        far = k % 2 == 1
        cx = float(rng.uniform(nx - 400, nx - 60) if far else rng.uniform(60, nx - 60))
        cy = float(rng.uniform(ny - 400, ny - 60) if far else rng.uniform(60, ny - 60))
        _paint_disk_window(mask, cx, cy, r, k + 1)
        rows.append([cx, cy, float(rng.uniform(-0.3, 0.3)) * u, float(rng.uniform(-0.3, 0.3)) * u,
                     float(rng.uniform(-1, 1)) * u / r])
    return Problem(name=f"huge{nx}x{ny}", nx=nx, ny=ny, tau_plus=tau_plus, magic_lambda=0.25, eta=1e-4,
                   bc=(INFLOW_EQ, OUTFLOW, PERIODIC, PERIODIC), rho_in=1.0, u_in=(u, 0.0),
                   body_force=(2e-5, -1e-5), mask=mask, bodies=np.array(rows), u_ref=u, l_ref=1.0)


def _nearest_image(c: np.ndarray, lo: int, n: int, period: int) -> np.ndarray:
    """Coordinates c relative to a cut starting at lo, taken at the periodic image
    nearest the cut's middle (a body past the wrap of the axis keeps its offsets
    to its own nodes)."""
    rel = c - lo
    return rel - period * np.round((rel - 0.5 * (n - 1)) / period)


def rows_band(p: Problem, j0: int, n: int) -> Problem:
    """Rows j0 .. j0 + n - 1 (taken modulo ny) of a problem as a problem of their
    own, periodic along y over the n rows, each body centre moved to band
    coordinates at its image nearest the band. A node update in the interior
    rows of a band reads that band only (the y sides are periodic)."""
    rs = [(j0 + s) % p.ny for s in range(n)]

    def cut(a):
        return None if a is None else np.ascontiguousarray(a[rs])

    b = p.bodies_or_empty().copy()
    b[:, 1] = _nearest_image(b[:, 1], j0, n, p.ny)
    return dataclasses.replace(p, name=f"{p.name}_rows{j0}+{n}", ny=n, mask=cut(p.mask_or_empty()),
                               bodies=b if b.shape[0] else None, rho_init=cut(p.rho_init),
                               ux_init=cut(p.ux_init), uy_init=cut(p.uy_init))


def split_x(p: Problem, widths: Sequence[int]) -> Tuple[List[Problem], List[int]]:
    """The slabs of a domain cut along x into consecutive column ranges of the
    given widths (summing to nx): each slab keeps its columns of the mask and of
    the initial fields and every body row with its centre moved to slab
    coordinates (cx - x0); cut sides become "neighbor", the domain's own x sides
    stay at the two ends (a periodic domain is cut there too). Returns the slab
    problems and their first columns x0."""
    if sum(widths) != p.nx or min(widths) < 3:
        raise ValueError("slab widths must be >= 3 and sum to nx")
    periodic = p.bc[0] == PERIODIC
    slabs, x0s = [], []
    x0 = 0
    for k, w in enumerate(widths):
        cols = slice(x0, x0 + w)
        west = "neighbor" if (k > 0 or periodic) else p.bc[0]
        east = "neighbor" if (k < len(widths) - 1 or periodic) else p.bc[1]
        b = p.bodies_or_empty().copy()
        b[:, 0] -= x0

        def cut(a):
            return None if a is None else np.ascontiguousarray(a[:, cols])

        slabs.append(dataclasses.replace(
            p, name=f"{p.name}_x{x0}+{w}", nx=w, bc=(west, east, p.bc[2], p.bc[3]), mask=cut(p.mask_or_empty()),
            bodies=b if b.shape[0] else None, rho_init=cut(p.rho_init), ux_init=cut(p.ux_init),
            uy_init=cut(p.uy_init)))
        x0s.append(x0)
        x0 += w
    return slabs, x0s
