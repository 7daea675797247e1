"""lbvp_batch_step_static, the batched step that allocates nothing (its tables
live in a static device array), against lbvp_batch_step through the C ABI:
populations, fields and force records bitwise equal, on two calls in a row on
different member sets, the second smaller than the first (the array keeps the
first call's tables, which the second must fully replace); tables beyond the
array's 4 MiB are rejected with E_ARG before anything runs."""
import numpy as np
import pytest
import torch

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")
PER = ("periodic",) * 4


def _big():
    mk = inputs.random_state_problem
    return [mk(300, 64, seed=151, n_disks=3, bc=IO, tau_plus=0.6),
            mk(67, 45, seed=152, n_disks=2, bc=IO),
            mk(1024, 33, seed=153, n_disks=4, bc=IO, body_force=(1e-5, 0.0)),
            mk(128, 128, seed=154, n_disks=2, bc=PER, tau_plus=0.9),
            mk(5, 7, seed=155, n_disks=1, bc=PER)]


def _small():
    mk = inputs.random_state_problem
    return [mk(61, 37, seed=156, n_disks=2, bc=IO), mk(40, 19, seed=157, n_disks=1, bc=PER)]


def _members(lbvp, probs, storage, flags, launch, stream):
    ms = [lbvp.Solver(p, storage=storage, force_every=1, force_capacity=128, flags=flags, stream=stream)
          for p in probs]
    for m in ms:
        m.set_launch(*launch)
    return ms


CASES = [("f32", False, (4, 256)), ("f16", False, (8, 128)), ("f64", True, (2, 64)), ("bf16", True, (1, 256))]


@pytest.mark.parametrize("storage,aa,launch", CASES, ids=[f"{s}-{'aa' if a else 'pull'}" for s, a, _ in CASES])
def test_static_batch_step_equals_the_batch(lbvp, storage, aa, launch):
    flags = lbvp.LAYOUT_AA if aa else 0
    for probs, steps in ((_big(), 36), (_small(), 12)):
        print(f"static batch {storage} aa={aa} launch={launch}: {len(probs)} members, {steps} steps", flush=True)
        stream = torch.cuda.Stream()
        st = _members(lbvp, probs, storage, flags, launch, stream)
        ref = _members(lbvp, probs, storage, flags, launch, stream)
        ctxs = [m.ctx for m in st]
        lbvp.lbvp_batch_step_static(ctxs, steps - 5, 0)
        lbvp.lbvp_batch_step_static(ctxs, 5, lbvp.KEEP_FIELDS)
        batch = lbvp.Batch(ref, vec=launch[0], block=launch[1])
        batch.step(steps - 5)
        batch.step(5, keep_fields=True)
        for p, a, b in zip(probs, st, ref):
            (fa, ma, sa), (fb, mb, sb) = a.forces(), b.forces()
            assert sa == sb == 1 and len(ma) == steps and np.all(np.isfinite(ma)), p.name
            assert np.array_equal(fa, fb) and np.array_equal(ma, mb), p.name
            fla, flb = a.fields(), b.fields()
            for k in fla:
                assert np.array_equal(fla[k], flb[k]), (p.name, k)
            assert np.array_equal(a.populations(), b.populations()), p.name
            assert a.step_count == b.step_count == steps
        batch.close()
        for m in st + ref:
            m.close()


def test_static_batch_step_rejects_what_it_cannot_hold(lbvp):
    stream = torch.cuda.Stream()
    # two 8192 x 4096 domains at one node per 64-thread block: 2 x 524288 tiles,
    # a tile map of 4 MiB on its own
    probs = [inputs.Problem(name=f"empty{k}", nx=8192, ny=4096, tau_plus=0.6, magic_lambda=0.25, eta=1e-4)
             for k in range(2)]
    ms = _members(lbvp, probs, "f16", lbvp.LAYOUT_AA, (1, 64), stream)
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_batch_step_static([m.ctx for m in ms], 2, 0)
    assert e.value.status == lbvp.E_ARG and "static array" in str(e.value)
    assert all(m.step_count == 0 for m in ms)
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_batch_step_static([ms[0].ctx], 2, lbvp.GRAPH)
    assert e.value.status == lbvp.E_ARG
    # one of them fits (2 MiB of tile map) and steps like lbvp_step
    lbvp.lbvp_batch_step_static([ms[0].ctx], 2, 0)
    ms[1].step(2)
    assert ms[0].step_count == 2 and np.array_equal(ms[0].populations(0, 3), ms[1].populations(0, 3))
    for m in ms:
        m.close()
