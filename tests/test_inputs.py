"""The seeded D3Q19 ensemble (inputs3.ensemble3) is what its recipe states:
deterministic, 64 sphere domains with sizes from the stated sets, one sphere
each inside its domain, Re and so tau+ in the stated range, 18,472,960 nodes
in all. Its lowest-tau+ domain stays bounded in the FP64 oracle over 300 steps
(the Re range was chosen for that; higher Re diverged within 600 steps).
"""
import numpy as np

from paper_1901_08766_amd import inputs3


def test_ensemble3_recipe():
    a, b = inputs3.ensemble3(), inputs3.ensemble3()
    assert len(a) == 64 and sum(p.n_nodes for p in a) == 18_472_960
    for p, q in zip(a, b):
        assert (p.nx, p.ny, p.nz, p.tau_plus) == (q.nx, q.ny, q.nz, q.tau_plus)
        assert np.array_equal(p.mask, q.mask) and np.array_equal(p.uy_init, q.uy_init)
    for p in a:
        assert p.nx in inputs3.ENSEMBLE3_NX and p.ny in inputs3.ENSEMBLE3_NYZ and p.nz in inputs3.ENSEMBLE3_NYZ
        assert p.bc == ("inflow_eq", "outflow_zero_grad") and p.n_bodies == 1
        assert 8.0 <= p.l_ref <= min(p.ny, p.nz) / 3.0
        re = p.u_ref * p.l_ref / ((p.tau_plus - 0.5) / 3.0)
        assert 20.0 - 1e-9 <= re <= 50.0 + 1e-9 and p.tau_plus >= 0.524
        solid = np.argwhere(p.mask == 1)
        assert len(solid) > 0 and solid.min() > 0 and (solid.max(axis=0) < [p.nz - 1, p.ny - 1, p.nx - 1]).all()
    assert len({(p.nx, p.ny, p.nz) for p in a}) > 10


def test_ensemble3_lowest_tau_domain_stays_bounded(ref3):
    probs = inputs3.ensemble3()
    p = min(probs, key=lambda q: (q.tau_plus, q.n_nodes))
    r = ref3.RefSolver3(p)
    _, mass = r.step(300, record=True)
    fl = r.fields()
    r.close()
    assert np.isfinite(mass).all() and abs(mass[-1] / p.n_nodes - 1.0) < 1e-3
    assert max(np.abs(fl[k]).max() for k in ("ux", "uy", "uz")) < 2.0 * p.u_ref
