"""Slab decomposition of one domain along x (LBVP_BC_NEIGHBOR sides and
lbvp_halo_exchange), on one GPU: the slabs, exchanged and stepped, must
reproduce the whole domain's step bitwise (populations and fields), and their
per-slab force and mass records must add up to the whole domain's. The whole
domain's step is itself the one the parity tests hold to the oracle.
"""
import numpy as np
import pytest

from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu


def _problem(nx, ny, seed, sides, n_disks=3):
    p = inputs.random_state_problem(nx, ny, seed=seed, n_disks=n_disks, bc=sides, body_force=(1e-5, -2e-6))
    # body centres on a 1/8 grid: moving them to slab coordinates is then exact
    # in both arithmetic types, so the obstacle velocities agree bitwise
    p.bodies[:, :2] = np.round(p.bodies[:, :2] * 8.0) / 8.0
    return p


def _whole_and_slabs(lbvp, p, widths, storage, steps, batched=True, launch=None):
    whole = lbvp.Solver(p, storage=storage, force_every=1, force_capacity=steps + 8)
    slabs_p, x0s = inputs.split_x(p, widths)
    slabs = lbvp.Slabs(slabs_p, x0s, storage=storage, force_every=1, force_capacity=steps + 8, batched=batched,
                       launch=launch)
    if launch is not None:
        whole.set_launch(*launch)
    print(f"case {p.name} widths={widths} storage={storage} steps={steps} batched={batched} launch={whole.launch}",
          flush=True)
    whole.step(steps, keep_fields=True)
    slabs.step(steps, keep_fields=True)
    return whole, slabs


PERIODIC = ("periodic",) * 4
INOUT = ("inflow_eq", "outflow_zero_grad", "periodic", "periodic")


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_self_linked_slab_is_the_periodic_domain(lbvp, storage):
    """One slab whose east cut feeds its own west cut steps bitwise like the
    periodic domain (every launch form: vector loads, lane shuffles)."""
    p = _problem(300, 37, 11, PERIODIC)
    whole, slabs = _whole_and_slabs(lbvp, p, [300], storage, 25)
    assert np.array_equal(whole.populations(), slabs.populations())
    slabs.close()
    whole.close()


CASES = [
    (INOUT, [20, 30, 17], 67, 45),
    (PERIODIC, [3, 64, 130, 103], 300, 23),
    (INOUT, [128, 128, 256, 512], 1024, 19),
]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("sides,widths,nx,ny", CASES, ids=["inout3", "periodic4", "inout4"])
def test_slabs_reproduce_the_whole_domain(lbvp, storage, sides, widths, nx, ny):
    p = _problem(nx, ny, 5, sides)
    steps = 30
    whole, slabs = _whole_and_slabs(lbvp, p, widths, storage, steps)
    assert np.array_equal(whole.populations(), slabs.populations())
    fw, fs = whole.fields(), slabs.fields()
    for k in fw:
        assert np.array_equal(fw[k], fs[k]), k
    gf, gm, _ = whole.forces()
    sf, sm = slabs.forces()
    tol = 1e-12 if storage == "f64" else 1e-6
    assert gf.shape == sf.shape and gm.shape == sm.shape
    scale = max(np.abs(gf).max(), 1e-30)
    assert np.abs(gf - sf).max() <= tol * scale
    assert np.abs(gm - sm).max() <= 1e-13 * gm.max()
    slabs.close()
    whole.close()


@pytest.mark.parametrize("launch", [(1, 64), (4, 256)], ids=["v1b64", "v4b256"])
def test_per_slab_launches_equal_the_batched_launch(lbvp, launch):
    p = _problem(300, 23, 7, INOUT)
    outs = []
    for batched in (True, False):
        whole, slabs = _whole_and_slabs(lbvp, p, [100, 101, 99], "f32", 20, batched=batched, launch=launch)
        outs.append(slabs.populations())
        assert np.array_equal(whole.populations(), outs[-1])
        slabs.close()
        whole.close()
    assert np.array_equal(outs[0], outs[1])


def test_halo_exchange_rejects_bad_links(lbvp):
    p = _problem(60, 20, 3, INOUT)
    slabs_p, x0s = inputs.split_x(p, [30, 30])
    slabs = lbvp.Slabs(slabs_p, x0s, storage="f32")
    a, b = slabs.solvers
    for west, east in ([a.ctx], [a.ctx]), ([b.ctx], [a.ctx]):   # a's west side is the inflow, b's east the outflow
        with pytest.raises(lbvp.LbvpError) as e:
            lbvp.lbvp_halo_exchange(west, east)
        assert e.value.status == lbvp.E_ARG
    other = lbvp.Solver(slabs_p[1], storage="f32")            # its own stream
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_halo_exchange([a.ctx], [other.ctx])
    assert e.value.status == lbvp.E_ARG
    lbvp.lbvp_halo_exchange([a.ctx], [b.ctx])
    other.close()
    slabs.close()


def test_graph_replays_of_the_slab_batch(lbvp):
    """The batched slabs captured in HIP graphs (halo kernels included) and
    replayed over calls, with plain calls between, stay bitwise on the whole
    domain's trajectory."""
    p = _problem(300, 23, 9, INOUT)
    whole = lbvp.Solver(p, storage="f32", force_every=1, force_capacity=128)
    slabs_p, x0s = inputs.split_x(p, [96, 120, 84])
    slabs = lbvp.Slabs(slabs_p, x0s, storage="f32", force_every=1, force_capacity=128)
    for k, (n, graph) in enumerate([(7, True), (7, True), (3, False), (7, True), (6, True)]):
        slabs.step(n, graph=graph)
        whole.step(n)
        slabs.forces()
        whole.forces()
        assert np.array_equal(whole.populations(), slabs.populations()), k
    slabs.close()
    whole.close()
