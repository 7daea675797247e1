"""The block -> tile order of the step kernels (lbvp_set_tile_band,
lbvp3_set_tile_band) only decides which workgroup updates which tile: every
order must give bitwise the same populations, fields and force and mass records.
The bands below cover whole groups with a ragged tail, a tail only (band past the
tiles one XCD holds) and plain dispatch order.
"""
import numpy as np
import pytest

from paper_1901_08766_amd import inputs, inputs3

pytestmark = pytest.mark.gpu

BANDS = [0, 1, 2, 8, 64, 65536]


def _run2(lbvp, prob, storage, launch, band, steps=25, flags=0):
    s = lbvp.Solver(prob, storage=storage, force_every=1, force_capacity=steps + 8, flags=flags)
    s.set_launch(*launch)
    s.set_tile_band(band)
    assert s.tile_band == band and s.launch == launch
    print(f"2-D {prob.nx}x{prob.ny} storage={storage} launch={launch} band={band}", flush=True)
    s.step(steps, keep_fields=True)
    out = (s.populations(), s.fields(), s.forces())
    s.close()
    return out


@pytest.mark.parametrize("storage,launch", [("f32", (4, 64)), ("f32", (1, 256)), ("f64", (2, 128)),
                                            ("f16", (8, 64)), ("bf16", (4, 128))])
def test_d2q9_tile_order_is_bitwise_neutral(lbvp, storage, launch):
    prob = inputs.random_state_problem(300, 41, seed=17, n_disks=4, body_force=(1e-5, -2e-6))
    ref = _run2(lbvp, prob, storage, launch, 0)
    for band in BANDS[1:]:
        pops, fields, (f, m, first) = _run2(lbvp, prob, storage, launch, band)
        assert np.array_equal(ref[0], pops), band
        for k in fields:
            assert np.array_equal(ref[1][k], fields[k]), (band, k)
        assert np.array_equal(ref[2][0], f) and np.array_equal(ref[2][1], m) and ref[2][2] == first, band


def test_d2q9_tile_order_aa_layout(lbvp):
    """In the in-place AA layout every slot is read and written by one node only,
    so the tile order cannot matter there either (both step parities; the state
    is read after an even count, where the layout holds it)."""
    prob = inputs.random_state_problem(300, 41, seed=19, n_disks=3,
                                       bc=("inflow_eq", "outflow_zero_grad", "periodic", "periodic"))
    ref = _run2(lbvp, prob, "f32", (4, 64), 0, steps=24, flags=lbvp.LAYOUT_AA)
    for band in (1, 8, 65536):
        pops, fields, (f, m, _) = _run2(lbvp, prob, "f32", (4, 64), band, steps=24, flags=lbvp.LAYOUT_AA)
        assert np.array_equal(ref[0], pops) and np.array_equal(ref[2][0], f) and np.array_equal(ref[2][1], m), band


def test_default_launches_take_bands(lbvp, lbvp3):
    """Large grids start with the measured vector shapes and bands; small ones
    with one node per thread and one eighth per XCD."""
    big = inputs.random_state_problem(2048, 1024, seed=1, n_disks=1)
    for storage, launch, band in (("f32", (4, 128), 8), ("f64", (2, 128), 2), ("f16", (4, 256), 16)):
        s = lbvp.Solver(big, storage=storage, force_every=0)
        assert (s.launch, s.tile_band) == (launch, band), storage
        s.close()
    s = lbvp.Solver(big, storage="f32", force_every=0, flags=lbvp.LAYOUT_AA)
    assert (s.launch, s.tile_band) == ((4, 128), 0)
    s.close()
    s3 = lbvp3.Solver3(inputs3.random_state_problem3(256, 128, 64, seed=1, n_spheres=1), storage="f16", force_every=0)
    assert (s3.launch, s3.tile_band) == ((4, 128), 4)
    s3.close()
    s = lbvp.Solver(inputs.random_state_problem(64, 40, seed=3, n_disks=1), storage="f32")
    assert s.tile_band == 0 and s.launch[0] == 1
    s.close()


def test_d2q9_tile_band_arguments(lbvp):
    prob = inputs.random_state_problem(64, 40, seed=3, n_disks=1)
    s = lbvp.Solver(prob, storage="f32")
    b0 = s.tile_band
    assert b0 == 0 or (b0 & (b0 - 1)) == 0
    for bad in (-1, 3, 12, 1 << 17):
        with pytest.raises(lbvp.LbvpError) as e:
            s.set_tile_band(bad)
        assert e.value.status == lbvp.E_ARG
    assert s.tile_band == b0
    s.set_tile_band(16)
    s.set_launch(1, 128)               # the band survives a new launch shape
    assert s.tile_band == 16
    s.close()


def _run3(lbvp3, prob, storage, launch, band, steps=12):
    s = lbvp3.Solver3(prob, storage=storage, force_every=1, force_capacity=steps + 8)
    s.set_launch(*launch)
    s.set_tile_band(band)
    assert s.tile_band == band
    print(f"3-D {prob.nx}x{prob.ny}x{prob.nz} storage={storage} launch={launch} band={band}", flush=True)
    s.step(steps, keep_fields=True)
    out = (s.populations(), s.fields(), s.forces())
    s.close()
    return out


@pytest.mark.parametrize("storage,launch", [("f32", (1, 64)), ("f32", (2, 128)), ("f64", (1, 128)),
                                            ("f16", (4, 64))])
def test_d3q19_tile_order_is_bitwise_neutral(lbvp3, storage, launch):
    prob = inputs3.random_state_problem3(72, 24, 20, seed=5, n_spheres=2)
    ref = _run3(lbvp3, prob, storage, launch, 0)
    for band in BANDS[1:]:
        pops, fields, (f, m, first) = _run3(lbvp3, prob, storage, launch, band)
        assert np.array_equal(ref[0], pops), band
        for k in fields:
            assert np.array_equal(ref[1][k], fields[k]), (band, k)
        assert np.array_equal(ref[2][0], f) and np.array_equal(ref[2][1], m) and ref[2][2] == first, band


def test_d3q19_tile_band_arguments(lbvp3):
    prob = inputs3.random_state_problem3(16, 12, 10, seed=2, n_spheres=1)
    s = lbvp3.Solver3(prob, storage="f32")
    b0 = s.tile_band
    for bad in (-2, 5, 1 << 20):
        with pytest.raises(lbvp3.LbvpError) as e:
            s.set_tile_band(bad)
        assert e.value.status == lbvp3.E_ARG
    assert s.tile_band == b0
    s.set_tile_band(4)
    s.set_launch(1, 64)
    assert s.tile_band == 4
    s.close()


def _batch_members():
    io = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")
    return [inputs.random_state_problem(128, 128, seed=41, n_disks=2, bc=io, tau_plus=0.55),
            inputs.random_state_problem(67, 45, seed=42, n_disks=3, bc=io, tau_plus=0.9),
            inputs.random_state_problem(300, 64, seed=44, n_disks=4, bc=("periodic",) * 4),
            inputs.random_state_problem(5, 7, seed=45, n_disks=1, bc=("periodic",) * 4),
            inputs.random_state_problem(1024, 33, seed=46, n_disks=2, bc=io)]


@pytest.mark.parametrize("storage,vec,aa", [("f32", 4, False), ("f16", 8, False), ("f32", 1, True)],
                         ids=["f32-pull", "f16-pull", "f32-aa"])
def test_batch_tile_order_is_bitwise_neutral(lbvp, storage, vec, aa):
    import torch
    flags = lbvp.LAYOUT_AA if aa else 0
    outs = []
    for band in (0, 1, 4, 64):
        stream = torch.cuda.Stream()
        members = [lbvp.Solver(p, storage=storage, force_every=1, force_capacity=64, flags=flags, stream=stream)
                   for p in _batch_members()]
        batch = lbvp.Batch(members, vec=vec, block=64)
        assert batch.tile_band == 0
        batch.set_tile_band(band)
        print(f"batch {storage} vec={vec} aa={aa} band={band}", flush=True)
        batch.step(9)
        batch.step(5, graph=True)
        batch.step(2, keep_fields=True)
        outs.append([(m.populations(), m.fields(), m.forces()) for m in members])
        batch.close()
        for m in members:
            m.close()
    for band, out in zip((1, 4, 64), outs[1:]):
        for (p0, f0, r0), (p1, f1, r1) in zip(outs[0], out):
            assert np.array_equal(p0, p1), band
            for k in f0:
                assert np.array_equal(f0[k], f1[k]), (band, k)
            assert np.array_equal(r0[0], r1[0]) and np.array_equal(r0[1], r1[1]) and r0[2] == r1[2], band


def test_batch_tile_band_arguments(lbvp):
    import torch
    stream = torch.cuda.Stream()
    members = [lbvp.Solver(p, storage="f32", stream=stream) for p in _batch_members()[:2]]
    batch = lbvp.Batch(members)
    for bad in (-1, 6, 1 << 18):
        with pytest.raises(lbvp.LbvpError) as e:
            batch.set_tile_band(bad)
        assert e.value.status == lbvp.E_ARG
    batch.set_tile_band(32)
    assert batch.tile_band == 32
    batch.close()
    for m in members:
        m.close()
