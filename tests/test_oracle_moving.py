"""The oracle's time-dependent mask (rigidly moving bodies), pinned to exact
kinematics and to the scheme's own invariants:

- bodies at rest (V = 0, omega = 0) reproduce the fixed-mask path bitwise;
- a translation by whole cells moves the mask by exactly those cells;
- a quarter turn of an asymmetric body about a node maps the mask to its
  90-degree rotation, and the turn's direction is counter-clockwise for omega > 0;
- a disk turning about its own centre keeps its mask away from the rim;
- on a periodic grid the total momentum changes each step by exactly the sum
  of the penalization forces of the nodes the bodies then cover;
- inside a moving body the corrected velocity satisfies the implicit
  penalization closed form about the body's velocity at its current position.
"""
import math

import numpy as np

from paper_1901_08766_amd import inputs


def _box(nx, ny, bodies, mask):
    p = inputs.random_state_problem(nx, ny, seed=3, n_disks=0, bc=("periodic",) * 4)
    p.mask = mask
    p.bodies = np.asarray(bodies, dtype=np.float64)
    p.moving = True
    return p


def _mask_at(s, nx, ny, t):
    return np.array([[s.body_at(i, j, t) for i in range(nx)] for j in range(ny)])


def test_bodies_at_rest_reproduce_the_fixed_path(oracle):
    runs = []
    for moving in (True, False):
        p = inputs.moving_bodies()
        p.bodies[:, 2:] = 0.0                  # V = 0, omega = 0
        p.moving = moving
        s = oracle.RefSolver(p)
        f, m = s.step(15, record=True)
        runs.append((s.populations(), f, m))
    (ga, fa, ma), (gb, fb, mb) = runs
    assert np.array_equal(ga, gb) and np.array_equal(fa, fb) and np.array_equal(ma, mb)


def test_translation_by_whole_cells(oracle):
    nx, ny = 40, 30
    mask = np.zeros((ny, nx), np.uint8)
    mask[10:14, 8:11] = 1                      # an asymmetric 3 x 4 block
    mask[12, 11] = 1
    s = oracle.RefSolver(_box(nx, ny, [[9.0, 11.5, 0.25, 0.5, 0.0]], mask))
    # at t = 4 the body has moved by (1, 2) cells
    moved = _mask_at(s, nx, ny, 4)
    expect = np.zeros_like(mask)
    expect[12:16, 9:12] = 1
    expect[14, 12] = 1
    assert np.array_equal(moved, expect)
    assert np.array_equal(_mask_at(s, nx, ny, 0), mask)


def test_quarter_turn_of_an_asymmetric_body(oracle):
    nx, ny = 41, 41
    c = 20
    mask = np.zeros((ny, nx), np.uint8)
    mask[c, c:c + 9] = 1                       # an arm along +x from the centre node
    mask[c:c + 3, c] = 1                       # and a short one along +y
    t = 10
    omega = (math.pi / 2) / t
    s = oracle.RefSolver(_box(nx, ny, [[float(c), float(c), 0.0, 0.0, omega]], mask))
    turned = _mask_at(s, nx, ny, t)
    # counter-clockwise by 90 degrees: +x arm -> +y arm, +y arm -> -x arm
    expect = np.zeros_like(mask)
    expect[c:c + 9, c] = 1
    expect[c, c - 2:c + 1] = 1
    assert np.array_equal(turned, expect)


def test_turning_disk_keeps_its_mask(oracle):
    nx, ny = 40, 40
    mask = np.zeros((ny, nx), np.uint8)
    inputs.paint_disk(mask, 19.3, 20.1, 8.4, 1)
    s = oracle.RefSolver(_box(nx, ny, [[19.3, 20.1, 0.0, 0.0, 0.013]], mask))
    ys, xs = np.mgrid[0:ny, 0:nx].astype(np.float64)
    rim = np.abs(np.hypot(xs - 19.3, ys - 20.1) - 8.4) < 1.0
    for t in (1, 7, 33):
        diff = _mask_at(s, nx, ny, t) != mask
        # nearest-node sampling of the turned disk can only change nodes next to the rim
        assert not (diff & ~rim).any()
        assert diff.sum() < 0.25 * rim.sum()


def _momentum(g, ex, ey):
    return np.array([(g * ex[:, None, None]).sum(), (g * ey[:, None, None]).sum()])


def test_momentum_budget_with_moving_bodies(oracle):
    p = inputs.moving_bodies(nx=160, ny=96)
    s = oracle.RefSolver(p)
    ex, ey, _, _ = oracle.lattice()
    n = p.nx * p.ny
    for _ in range(4):
        P0 = _momentum(s.populations(), ex, ey)
        f, _ = s.step(1, record=True)
        fl = s.fields()
        P1 = _momentum(s.populations(), ex, ey)
        F = np.array([fl["fx"].sum(), fl["fy"].sum()])
        assert np.abs(P1 - P0 - F).max() <= 1e-13 * n * 0.1
        # the records are minus the same sums, split over the bodies
        assert np.abs(f[0].sum(axis=0) + F).max() <= 1e-12 * max(1.0, np.abs(F).max())


def test_penalized_velocity_follows_the_moving_body(oracle):
    """Inside body b at time level t the corrected velocity u and the
    intermediate u* obey u - U_O = (u* - U_O) 2 eta / (2 eta + 1), with
    U_O = V + omega z x (x - c(t)); with F_VP = 2 rho (u - u*) this reads
    F_VP = 2 rho (U_O - u*) / (2 eta + 1), checked through u - U_O = -F_VP eta / rho."""
    p = inputs.moving_bodies(nx=160, ny=96)
    s = oracle.RefSolver(p)
    s.step(12)
    t = 12
    fl = s.fields()
    ys, xs = np.mgrid[0:p.ny, 0:p.nx].astype(np.float64)
    ids = _mask_at(s, p.nx, p.ny, t)
    checked = 0
    for b in range(1, p.n_bodies + 1):
        cx, cy, vx, vy, om = p.bodies[b - 1]
        cxt, cyt = cx + vx * t, cy + vy * t
        sel = ids == b
        uox = vx - om * (ys[sel] - cyt)
        uoy = vy + om * (xs[sel] - cx - vx * t)
        rho = fl["rho"][sel]
        assert np.abs(fl["ux"][sel] - uox + fl["fx"][sel] * p.eta / rho).max() <= 1e-14
        assert np.abs(fl["uy"][sel] - uoy + fl["fy"][sel] * p.eta / rho).max() <= 1e-14
        checked += sel.sum()
    assert checked > 200
