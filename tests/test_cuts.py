"""The sampled checks of large domains cut a band of rows (2-D) or a slab of
planes (3-D) out of the domain and let the oracle advance its interior by one
step. These cuts must not change what the oracle computes there: on small
domains, stepping the band's interior rows gives exactly the whole domain's
step at those nodes (bodies near the cut, the wrap of the periodic axis, and
inflow/outflow columns included), and the cut itself keeps the mask, bodies
and initial fields of the rows it takes.
"""
import dataclasses

import numpy as np

from paper_1901_08766_amd import inputs, inputs3

IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")


def test_rows_band_takes_rows_modulo_ny(oracle):
    p = inputs.random_state_problem(23, 17, seed=4, n_disks=3, bc=IO)
    b = inputs.rows_band(p, 15, 5)                  # rows 15, 16, 0, 1, 2
    rows = [15, 16, 0, 1, 2]
    assert b.ny == 5 and b.nx == p.nx and b.bc == p.bc
    assert np.array_equal(b.mask, p.mask[rows]) and np.array_equal(b.ux_init, p.ux_init[rows])
    assert np.array_equal(b.bodies[:, 1], p.bodies[:, 1] - 15)
    assert np.array_equal(b.bodies[:, [0, 2, 3, 4]], p.bodies[:, [0, 2, 3, 4]])


def _on_eighths(bodies, cols):
    """Body centres on a 1/8 grid: moving them by whole rows or planes is then
    exact in FP64, so offsets from the centre agree bitwise after a cut."""
    b = bodies.copy()
    b[:, cols] = np.round(b[:, cols] * 8.0) / 8.0
    return b


def _edge_bodies(p):
    """The problem with two rotating, translating disks added against the first
    and the last row, so that cuts across the wrap of y hold their nodes."""
    mask = p.mask.copy()
    rows = [_on_eighths(p.bodies, [0, 1])]
    for k, (cx, cy) in enumerate([(11.375, 0.625), (27.75, p.ny - 1.375)]):
        inputs.paint_disk(mask, cx, cy, 3.7, p.n_bodies + 1 + k)
        rows.append(np.array([[cx, cy, 0.01, -0.004, 0.003 * (1 - 2 * k)]]))
    return dataclasses.replace(p, mask=mask, bodies=np.concatenate(rows))


def test_band_interior_steps_like_the_whole_domain(oracle):
    # disks of radius up to 4 on a 40 x 24 grid, two against the wrap of y
    p = _edge_bodies(inputs.random_state_problem(40, 24, seed=12, n_disks=4, bc=IO, body_force=(1e-5, -3e-6)))
    assert (p.mask[0] == 5).any() and (p.mask[-1] == 6).any()
    whole = oracle.RefSolver(p)
    whole.step(3)
    g = whole.populations()
    for lo, n in [(22, 4), (0, 3), (9, 7), (23, 3), (20, 8), (22, 3)]:
        band = inputs.rows_band(p, lo, n)
        ref = oracle.RefSolver(band)
        gb = np.ascontiguousarray(g[:, [(lo + s) % p.ny for s in range(n)]])
        ys = np.repeat(np.arange(1, n - 1), p.nx)
        xs = np.tile(np.arange(p.nx), n - 2)
        got, fl = ref.step_nodes(gb, xs, ys)
        want, wfl = whole.step_nodes(g, xs, (ys + lo) % p.ny)
        assert np.array_equal(got, want), (lo, n)
        assert np.array_equal(fl, wfl), (lo, n)
        ref.close()
    whole.close()


def test_slab_interior_steps_like_the_whole_domain(ref3):
    p = inputs3.random_state_problem3(14, 10, 9, seed=6, n_spheres=3, body_force=(1e-5, 0.0, -2e-6))
    mask = p.mask.copy()                                # a turning sphere against the first plane
    inputs3.paint_sphere(mask, 6.25, 4.75, 0.75, 2.6, p.n_bodies + 1)
    row = np.array([[6.25, 4.75, 0.75, 0.01, 0.0, -0.005, 0.002, -0.003, 0.004]])
    p = dataclasses.replace(p, mask=mask, bodies=np.concatenate([_on_eighths(p.bodies, [0, 1, 2]), row]))
    assert (p.mask[0] == p.n_bodies).any()
    whole = ref3.RefSolver3(p)
    whole.step(2)
    g = whole.populations()
    for k0 in (8, 0, 3, 7):
        slab = inputs3.slab(p, k0, 3)
        ref = ref3.RefSolver3(slab)
        gs = np.ascontiguousarray(g[:, [(k0 + s) % p.nz for s in range(3)]])
        ys, xs = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
        xs, ys = xs.ravel(), ys.ravel()
        got, fl = ref.step_nodes(gs, xs, ys, np.ones_like(xs))
        want, wfl = whole.step_nodes(g, xs, ys, np.full_like(xs, (k0 + 1) % p.nz))
        assert np.array_equal(got, want), k0
        assert np.array_equal(fl, wfl), k0
        ref.close()
    whole.close()
