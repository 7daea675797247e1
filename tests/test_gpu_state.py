"""Checkpoint and resume (lbvp_save_state / lbvp_load_state): a context restored
from a saved state continues bitwise as the saved one would have (populations,
fields, force records), in both layouts and at either step parity."""
import numpy as np
import pytest

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

SIDES_IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")


@pytest.mark.parametrize("storage,aa,first", [("f32", False, 37), ("f32", True, 37), ("f32", True, 36),
                                              ("f16", True, 21), ("f64", False, 10), ("bf16", False, 9)])
def test_resume_is_bitwise(lbvp, storage, aa, first):
    flags = lbvp.LAYOUT_AA if aa else 0
    prob = inputs.random_state_problem(150, 70, seed=61, n_disks=3, bc=SIDES_IO)
    a = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=256, flags=flags)
    a.step(first, keep_fields=True)
    a.forces()
    blob = a.save_state()
    print(f"state {storage} aa={aa} after {first} steps: {blob.nbytes} bytes", flush=True)
    b = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=256, flags=flags)
    b.step(5)                      # some other history first: the load replaces it
    b.forces()
    b.load_state(blob)
    assert b.step_count == first
    fa0, fb0 = a.fields(), b.fields()
    for k in fa0:
        assert np.array_equal(fa0[k], fb0[k]), k
    a.step(25, keep_fields=True)
    b.step(25, keep_fields=True)
    (ga, ma, sa), (gb, mb, sb) = a.forces(), b.forces()
    assert sa == sb == first + 1 and np.array_equal(ga, gb) and np.array_equal(ma, mb)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    if not aa or (first + 25) % 2 == 0:
        assert np.array_equal(a.populations(), b.populations())


def test_state_rejections(lbvp):
    prob = inputs.random_state_problem(64, 40, seed=62, n_disks=1, bc=SIDES_IO)
    a = lbvp.Solver(prob, storage="f32", force_every=1, force_capacity=64)
    a.step(3)
    with pytest.raises(lbvp.LbvpError) as e:         # undrained records
        a.save_state()
    assert e.value.status == lbvp.E_STATE
    a.forces()
    blob = a.save_state()
    other = inputs.random_state_problem(64, 41, seed=62, n_disks=1, bc=SIDES_IO)
    for p2, st, fl in ((other, "f32", 0), (prob, "f16", 0), (prob, "f32", lbvp.LAYOUT_AA)):
        c = lbvp.Solver(p2, storage=st, force_every=1, force_capacity=64, flags=fl)
        with pytest.raises(lbvp.LbvpError) as e:
            c.load_state(blob)
        assert e.value.status == lbvp.E_ARG
        c.close()
    bad = blob.copy()
    bad[0] ^= 0xFF
    with pytest.raises(lbvp.LbvpError):
        a.load_state(bad)
    with pytest.raises(lbvp.LbvpError):
        a.load_state(blob[:100])
