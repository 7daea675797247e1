"""LBVP_PERSISTENT: a run of batched steps as one cooperative launch with a grid
barrier between steps must give bitwise the results of the plain batched call
(one launch per step): populations, fields of the last step and every force
and mass record, for records every step and every third step, several calls
in a row (lattice parity and record phase carried across calls)."""
import numpy as np
import pytest
import torch

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

SIDES_IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")
SIDES_P = ("periodic",) * 4


def _members():
    mk = inputs.random_state_problem
    return [mk(128, 128, seed=161, n_disks=2, bc=SIDES_IO, tau_plus=0.55),
            mk(67, 45, seed=162, n_disks=3, bc=SIDES_IO, tau_plus=0.9),
            mk(256, 19, seed=163, n_disks=1, bc=SIDES_P, body_force=(1e-5, 0.0)),
            mk(1024, 33, seed=164, n_disks=4, bc=("outflow_zero_grad", "inflow_eq", "periodic", "periodic")),
            mk(5, 7, seed=165, n_disks=1, bc=SIDES_P)]


def _run(lbvp, probs, storage, launch, force_every, persistent, calls):
    stream = torch.cuda.Stream()
    ms = [lbvp.Solver(p, storage=storage, force_every=force_every, force_capacity=256, stream=stream) for p in probs]
    b = lbvp.Batch(ms, vec=launch[0], block=launch[1])
    for n, keep in calls:
        b.step(n, keep_fields=keep, persistent=persistent)
    out = []
    for m in ms:
        f, mass, first = m.forces()
        out.append((f, mass, first, m.fields(), m.populations(), m.step_count))
    b.close()
    for m in ms:
        m.close()
    return out


@pytest.mark.parametrize("storage,launch", [("f32", (4, 128)), ("f32", (1, 256)), ("f16", (4, 256)),
                                            ("bf16", (8, 64)), ("f64", (2, 128))])
@pytest.mark.parametrize("force_every", [1, 3])
def test_persistent_equals_plain_batch(lbvp, storage, launch, force_every):
    probs = _members()
    calls = [(7, False), (1, False), (12, True)]
    print(f"persistent {storage} launch={launch} force_every={force_every}", flush=True)
    a = _run(lbvp, probs, storage, launch, force_every, False, calls)
    b = _run(lbvp, probs, storage, launch, force_every, True, calls)
    for p, x, y in zip(probs, a, b):
        fx, mx, sx, flx, gx, nx = x
        fy, my, sy, fly, gy, ny = y
        assert nx == ny == 20 and sx == sy
        assert len(mx) == 20 // force_every and np.all(np.isfinite(mx))
        assert np.array_equal(fx, fy) and np.array_equal(mx, my), p.name
        for k in flx:
            assert np.array_equal(flx[k], fly[k]), (p.name, k)
        assert np.array_equal(gx, gy), p.name


def test_persistent_rejections(lbvp):
    probs = _members()[:2]
    stream = torch.cuda.Stream()
    aa = [lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64, flags=lbvp.LAYOUT_AA, stream=stream)
          for p in probs]
    b = lbvp.Batch(aa)
    with pytest.raises(lbvp.LbvpError) as e:
        b.step(2, persistent=True)
    assert e.value.status == lbvp.E_ARG
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_step(aa[0].ctx, 2, lbvp.PERSISTENT)
    assert e.value.status == lbvp.E_ARG
    b.close()
    pull = [lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64, stream=stream) for p in probs]
    b = lbvp.Batch(pull)
    with pytest.raises(lbvp.LbvpError) as e:
        b.step(2, graph=True, persistent=True)
    assert e.value.status == lbvp.E_ARG
    b.step(2, persistent=True)
    assert all(m.step_count == 2 for m in pull)
    b.close()
