"""The serving pool (continuous batching): solves admitted at different times,
with different sizes, bodies and step counts, overlap on the device; each result
(force and mass records of every step, final fields) must be bitwise that of the
same problem stepped alone with the pool's launch shape. Also the tuner."""
import numpy as np
import pytest
import torch

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

SIDES_IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")
VW = {"f64": 2, "f32": 4, "f16": 8, "bf16": 8}


def _requests():
    """(problem, steps, admitted before epoch k)."""
    mk = inputs.random_state_problem
    return [
        (mk(128, 64, seed=81, n_disks=2, bc=SIDES_IO, tau_plus=0.6), 57, 0),
        (mk(67, 45, seed=82, n_disks=1, bc=SIDES_IO, tau_plus=0.8), 23, 0),
        (mk(256, 32, seed=83, n_disks=3, bc=SIDES_IO), 90, 1),
        (mk(40, 40, seed=84, n_disks=0, bc=("periodic",) * 4), 11, 2),
        (mk(300, 50, seed=85, n_disks=2, bc=SIDES_IO), 40, 4),
        (mk(96, 96, seed=86, n_disks=4, bc=SIDES_IO), 1, 5),
        (mk(64, 33, seed=87, n_disks=1, bc=SIDES_IO), 33, 5),
    ]


def _alone(lbvp, prob, steps, storage, flags, vec, block):
    s = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=steps + 1, flags=flags)
    s.set_launch(vec, block)
    s.step(steps, keep_fields=True)
    forces, mass, first = s.forces()
    fields = s.fields()
    s.close()
    return forces, mass, first, fields


@pytest.mark.parametrize("storage,aa", [("f32", False), ("f32", True), ("f16", False), ("bf16", True),
                                        ("f64", False)])
def test_each_result_is_the_same_alone_and_in_the_mix(lbvp, storage, aa):
    flags = lbvp.LAYOUT_AA if aa else 0
    vec = 1 if (aa and storage in ("f16", "bf16")) else VW[storage]
    block = 128
    pool = lbvp.Pool(storage=storage, layout_aa=aa, cap_bytes=1 << 30, max_slots=4, vec=vec, block=block,
                     chunk_bytes=64 << 20, max_in_flight=2)
    reqs = _requests()
    pending = list(range(len(reqs)))
    slot_of, results = {}, {}
    epoch = 0
    while pending or slot_of:
        for k in list(pending):
            prob, steps, at = reqs[k]
            if at > epoch:
                continue
            slot = pool.admit(prob, steps)
            if slot is None:
                break          # full: retried after a completion (FIFO)
            slot_of[slot] = k
            pending.remove(k)
        ran = pool.run_epoch(16)
        epoch += 1
        for slot in pool.poll(wait=(ran == 0)):
            k = slot_of.pop(slot)
            f, m, first = pool.forces(slot)
            results[k] = (f, m, first, pool.fields(slot))
            pool.release(slot)
        assert epoch < 500
    st = pool.stats()
    assert st["free_slots"] == 4 and st["used_bytes"] == 0 and st["running"] == 0
    assert st["node_updates"] == sum(p.nx * p.ny * n for p, n, _ in reqs)
    pool.close()
    for k, (prob, steps, _) in enumerate(reqs):
        print(f"pool {storage} aa={aa} request {k} {prob.nx}x{prob.ny} {steps} steps", flush=True)
        f, m, first, fields = results[k]
        fa, ma, firsta, fieldsa = _alone(lbvp, prob, steps, storage, flags, vec, block)
        assert len(m) == steps and first == firsta == 1
        assert np.array_equal(f, fa) and np.array_equal(m, ma), k
        for name in fields:
            assert np.array_equal(fields[name], fieldsa[name]), (k, name)


def test_admission_limits(lbvp):
    stream = torch.cuda.Stream()
    small = inputs.random_state_problem(64, 32, seed=91, n_disks=1, bc=SIDES_IO)
    params = lbvp.params_for(small, "f32", 1, 101, max_bodies=1)
    fp = lbvp.lbvp_footprint_bytes(params)
    # slots
    pool = lbvp.Pool(storage="f32", cap_bytes=1 << 30, max_slots=2, stream=stream)
    a, b = pool.admit(small, 100), pool.admit(small, 100)
    assert a is not None and b is not None and pool.admit(small, 100) is None
    pool.release(a)                       # not started yet: may be released
    c = pool.admit(small, 100)
    assert c is not None
    pool.close()
    # memory: room for two solves under the cap, not three
    pool = lbvp.Pool(storage="f32", cap_bytes=2 * fp + 4096, max_slots=8, chunk_bytes=1, stream=stream)
    s1, s2 = pool.admit(small, 100), pool.admit(small, 100)
    assert s1 is not None and s2 is not None and pool.admit(small, 100) is None
    assert pool.stats()["used_bytes"] <= 2 * fp + 4096
    while pool.run_epoch(64):
        pass
    done = set()
    while len(done) < 2:
        done.update(pool.poll(wait=True))
    for s in done:
        pool.release(s)
    s3 = pool.admit(small, 100)
    assert s3 is not None
    # a running solve cannot be released; wrong storage is rejected
    assert pool.run_epoch(10) == 10
    with pytest.raises(lbvp.LbvpError) as e:
        pool.release(s3)
    assert e.value.status == lbvp.E_STATE
    pool16 = lbvp.Pool(storage="f16", cap_bytes=1 << 28, max_slots=2, stream=stream)
    with pytest.raises(lbvp.LbvpError):
        lbvp.lbvp_pool_admit(pool16.handle, params, small.mask_or_empty(), small.bodies_or_empty(), n_steps=5)
    pool16.close()
    pool.close()


def test_tuner_measures_every_shape_and_leaves_members_alone(lbvp):
    stream = torch.cuda.Stream()
    probs = [inputs.random_state_problem(256, 128, seed=95 + k, n_disks=2, bc=SIDES_IO) for k in range(3)]
    members = [lbvp.Solver(p, storage="f32", force_every=1, force_capacity=64, stream=stream) for p in probs]
    for m in members:
        m.step(5)
    before = [m.populations() for m in members]
    rows, best = lbvp.tune(members, steps=20, layouts=True, fresh=True)
    shapes = {(r["layout_flags"], r["vec"], r["block"], r["band"]) for r in rows}
    assert len(shapes) == len(rows)
    assert shapes == {(l, v, b, t) for l in (0, lbvp.LAYOUT_AA) for v in (1, 4) for b in (64, 128, 256)
                      for t in ((0,) if v == 1 else (0, 2, 16))}
    assert all(r["ms_per_step"] > 0 and r["mlups"] > 0 for r in rows)
    fastest = min(r["ms_per_step"] for r in rows)
    assert best["ms_per_step"] <= 1.03 * fastest + 1e-12
    for m, g in zip(members, before):
        assert m.step_count == 5 and np.array_equal(m.populations(), g)
    rows2, best2 = lbvp.tune(members, steps=20, layouts=True)     # from the cache
    assert rows2 == rows and best2 == best
    for m in members:
        m.forces()                                                  # drained: the shape may change
    batch = lbvp.Batch(members, vec=best["vec"], block=best["block"])
    batch.set_tile_band(best["band"])
    batch.step(3)
    batch.close()


def test_served_stream_results_equal_alone(lbvp):
    """The serving loop (arrivals on the clock, FIFO admission, epochs, hand-off)
    on a short stream of small requests: every served result equals the same
    solve run alone."""
    from paper_1901_08766_amd import serve

    reqs = inputs.request_stream(rate=400.0, n=10, seed=11, step_lo=20, step_hi=300, sizes=[(128, 64), (96, 48)])
    pool = lbvp.Pool(storage="f32", cap_bytes=1 << 30, max_slots=3, vec=4, block=256, chunk_bytes=32 << 20)
    got = {}
    rep = serve.serve(reqs, pool, max_epoch_steps=64, fields=True,
                      on_result=lambda r, f, m, fl: got.__setitem__(r.rid, (f, m, fl)))
    pool.close()
    assert sorted(got) == list(range(10)) and not rep.unstable
    assert rep.max_resident <= 3 and rep.percentile(99) >= rep.percentile(50) > 0
    for r in reqs:
        f, m, fl = got[r.rid]
        fa, ma, _, fla = _alone(lbvp, r.problem, r.problem.steps, "f32", 0, 4, 256)
        assert np.array_equal(f, fa) and np.array_equal(m, ma), r.rid
        for k in fl:
            assert np.array_equal(fl[k], fla[k]), (r.rid, k)
