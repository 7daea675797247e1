"""Step sequences enqueued through HIP graphs (LBVP_GRAPH) and the record sums'
independence of how steps are split over calls. Every graph replay is checked
against the same steps enqueued as plain launches, with plain work and host
synchronisations between the replays; the replays must be bitwise equal."""
import numpy as np
import pytest
import torch

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

SIDES_IO = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")


def _prob(nx=96, ny=40, seed=71):
    return inputs.random_state_problem(nx, ny, seed=seed, n_disks=2, bc=SIDES_IO, tau_plus=0.6)


def _same(a, b, what):
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), (what, k)
    (ga, ma, sa), (gb, mb, sb) = a.forces(), b.forces()
    assert sa == sb and np.array_equal(ga, gb) and np.array_equal(ma, mb), what
    assert a.step_count == b.step_count, what


@pytest.mark.parametrize("aa", [False, True], ids=["pull", "aa"])
@pytest.mark.parametrize("force_every", [1, 3])
def test_graph_replays_equal_plain_launches(lbvp, aa, force_every):
    flags = lbvp.LAYOUT_AA if aa else 0
    p = _prob()
    plain = lbvp.Solver(p, storage="f32", force_every=force_every, force_capacity=4096, flags=flags)
    graph = lbvp.Solver(p, storage="f32", force_every=force_every, force_capacity=4096, flags=flags)
    # odd and even call lengths, one longer than a captured chunk (512 steps)
    for rep, n in enumerate([7, 7, 6, 7, 1030, 7, 1030]):
        print(f"graph aa={aa} fe={force_every} call {rep}: {n} steps", flush=True)
        plain.step(n, keep_fields=True)
        graph.step(n, keep_fields=True, graph=True)
        plain.synchronize()
        graph.synchronize()
        _same(plain, graph, f"call {rep}")
        if not aa or plain.step_count % 2 == 0:
            assert np.array_equal(plain.populations(), graph.populations()), rep
        # plain work on the graph's context between replays
        plain.step(2)
        graph.step(2)
    plain.close()
    graph.close()


def test_records_do_not_depend_on_call_splitting(lbvp):
    p = _prob(seed=72)
    one = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=512)
    split = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=512)
    one.step(40, keep_fields=True)
    for n in (1, 2, 3, 5, 8, 21):
        split.step(n, keep_fields=(n == 21))
    _same(one, split, "split")


@pytest.mark.parametrize("block", [64, 128])
def test_record_sums_do_not_depend_on_block_of_the_summing_launch(lbvp, block):
    """The record of step k is summed by tile 0 of step k + 1 (a block of the step
    launch) or by the standalone finalize (256 threads): same bits."""
    p = _prob(seed=73)
    a = lbvp.Solver(p, storage="f64", force_every=1, force_capacity=512)
    b = lbvp.Solver(p, storage="f64", force_every=1, force_capacity=512)
    a.set_launch(1, block)
    b.set_launch(1, block)
    a.step(30)
    for _ in range(30):
        b.step(1)
    (ga, ma, _), (gb, mb, _) = a.forces(), b.forces()
    assert np.array_equal(ga, gb) and np.array_equal(ma, mb)


@pytest.mark.parametrize("aa", [False, True], ids=["pull", "aa"])
def test_batch_graph_replays_equal_plain_batch(lbvp, aa):
    flags = lbvp.LAYOUT_AA if aa else 0
    probs = [_prob(96, 40, 74), _prob(64, 64, 75), _prob(200, 17, 76)]
    sp, sg = torch.cuda.Stream(), torch.cuda.Stream()
    mp = [lbvp.Solver(q, storage="f32", force_every=1, force_capacity=4096, flags=flags, stream=sp) for q in probs]
    mg = [lbvp.Solver(q, storage="f32", force_every=1, force_capacity=4096, flags=flags, stream=sg) for q in probs]
    bp, bg = lbvp.Batch(mp), lbvp.Batch(mg)
    for rep, n in enumerate([5, 5, 4, 600, 5]):
        print(f"batch graph aa={aa} call {rep}: {n} steps", flush=True)
        bp.step(n, keep_fields=True)
        bg.step(n, keep_fields=True, graph=True)
        for a, b in zip(mp, mg):
            a.synchronize()
            b.synchronize()
            _same(a, b, f"call {rep}")
        bp.step(2)
        bg.step(2)
    bp.close()
    bg.close()


def test_graph_rejects_the_null_stream(lbvp):
    p = _prob(seed=77)
    s = lbvp.Solver(p, storage="f32", stream=torch.cuda.default_stream())
    if s.stream.cuda_stream != 0:
        pytest.skip("torch's default stream is not the null stream here")
    with pytest.raises(lbvp.LbvpError) as e:
        s.step(3, graph=True)
    assert e.value.status == lbvp.E_ARG
    s.close()
