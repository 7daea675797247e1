"""Moving bodies (LBVP_MOVING_BODIES, a time-dependent mask) through the C ABI
against the oracle's independent implementation: node membership is evaluated
in FP64 on both sides the same way, so FP64 runs agree to 1e-12 including the
steps where nodes switch between fluid and solid."""
import numpy as np
import pytest
import torch

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

SIDES_IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("sides,u_in,steps", [(("periodic",) * 4, 0.0, 40), (SIDES_IO, 0.03, 40),
                                              (("periodic",) * 4, 0.0, 1100)],
                         ids=["periodic", "inflow-outflow", "past-one-pose-table"])
def test_fp64_matches_oracle(lbvp, oracle, sides, u_in, steps):
    p = inputs.moving_bodies(bc=sides, u_in=u_in)
    g = lbvp.Solver(p, storage="f64", force_every=1, force_capacity=steps + 8)
    print(f"moving {p.name} sides={sides[0]}/{sides[1]} {steps} steps", flush=True)
    g.step(steps, keep_fields=True)
    gf, gm, first = g.forces()
    r = oracle.RefSolver(p)
    rf, rm = r.step(steps, record=True)
    tol = 1e-12 if steps < 100 else 1e-11
    assert _rel(g.populations(), r.populations()) <= tol
    fa, fr = g.fields(), r.fields()
    for k in fa:
        assert np.abs(fa[k] - fr[k]).max() <= tol * max(1.0, np.abs(fr[k]).max()), k
    scale = np.abs(fr["fx"]).sum() + np.abs(fr["fy"]).sum()
    assert first == 1 and np.abs(gf - rf).max() <= tol * scale
    assert np.abs(gm - rm).max() <= 1e-13 * rm.max()


def test_fp32_matches_oracle(lbvp, oracle):
    p = inputs.moving_bodies()
    g = lbvp.Solver(p, storage="f32", force_every=0)
    g.step(300, keep_fields=True)
    r = oracle.RefSolver(p)
    r.step(300)
    a, b = g.fields(), r.fields()
    err = np.sqrt(np.sum((a["ux"] - b["ux"]) ** 2 + (a["uy"] - b["uy"]) ** 2) / np.sum(b["ux"] ** 2 + b["uy"] ** 2))
    print(f"moving fp32 velocity rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("steps", [17, 18])
def test_aa_equals_pull(lbvp, steps):
    p = inputs.moving_bodies(bc=SIDES_IO, u_in=0.03)
    a = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64)
    b = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64, flags=lbvp.LAYOUT_AA)
    a.step(steps, keep_fields=True)
    b.step(steps, keep_fields=True)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    (ga, ma, _), (gb, mb, _) = a.forces(), b.forces()
    assert np.array_equal(ga, gb) and np.array_equal(ma, mb)
    if steps % 2 == 0:
        assert np.array_equal(a.populations(), b.populations())


def test_bodies_at_rest_equal_the_fixed_mask(lbvp):
    outs = []
    for moving in (True, False):
        p = inputs.moving_bodies()
        p.bodies[:, 2:] = 0.0
        p.moving = moving
        s = lbvp.Solver(p, storage="f64", force_every=1, force_capacity=64)
        s.set_launch(1, 64)
        s.step(25)
        f, m, _ = s.forces()
        outs.append((s.populations(), f, m))
    (ga, fa, ma), (gb, fb, mb) = outs
    assert np.array_equal(ga, gb) and np.array_equal(ma, mb)
    # the per-body sums run over differently laid out partial lists: last bits only
    assert np.abs(fa - fb).max() <= 1e-14 * max(np.abs(fb).max(), 1e-300) * 10


def test_moving_rejections(lbvp):
    p = inputs.moving_bodies()
    s = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64, stream=torch.cuda.Stream())
    with pytest.raises(lbvp.LbvpError) as e:
        s.step(2, graph=True)
    assert e.value.status == lbvp.E_ARG
    with pytest.raises(lbvp.LbvpError):
        s.set_launch(4, 256)
    q = inputs.random_state_problem(64, 32, seed=5, n_disks=1)
    other = lbvp.Solver(q, storage="f32", force_every=1, force_capacity=64, stream=s.stream)
    with pytest.raises(lbvp.LbvpError):
        lbvp.Batch([s, other])
    pool = lbvp.Pool(storage="f32", cap_bytes=1 << 28, max_slots=2, stream=s.stream)
    params = lbvp.params_for(p, "f32", 1, 0)
    with pytest.raises(lbvp.LbvpError):
        lbvp.lbvp_pool_admit(pool.handle, params, p.mask_or_empty(), p.bodies_or_empty(), n_steps=3)
    pool.close()
