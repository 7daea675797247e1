"""The benchmark's algorithmic byte count (host only): the mask byte is counted
for exactly the nodes of tiles that hold a solid node, with the tiling the
library's launch shapes make (D2Q9 tile width a power of two up to vec x
block, D3Q19 nx rounded up to vec)."""
import importlib.util
import os

import numpy as np
import pytest

from paper_1901_08766_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("nx,ny,launch", [(67, 45, (1, 64)), (300, 41, (4, 64)), (130, 70, (4, 256)),
                                          (1024, 33, (2, 128)), (5, 7, (1, 256))])
def test_mask_fraction_by_brute_force(bench, nx, ny, launch):
    p = inputs.random_state_problem(nx, ny, seed=nx + ny, n_disks=2)
    vec, block = launch
    tw, tr = bench.tile_shape(nx, {"vec": vec, "block": block})
    assert tw * tr == vec * block and tw & (tw - 1) == 0 and tw >= vec
    assert tw == min(vec * block, max(vec, 1 << max(nx - 1, 0).bit_length()))
    count = 0
    for j0 in range(0, ny, tr):
        for i0 in range(0, nx, tw):
            tile = p.mask[j0:j0 + tr, i0:i0 + tw]
            if (tile > 0).any():
                count += tile.size
    got = bench.mask_read_fraction(p, {"vec": vec, "block": block})
    assert got == pytest.approx(count / (nx * ny), abs=0, rel=1e-15)
    assert bench.alg_bytes_per_node("f32", p, {"vec": vec, "block": block}) == 72 + got


def test_no_bodies_reads_no_mask(bench):
    p = inputs.random_state_problem(64, 32, seed=3, n_disks=0)
    assert bench.mask_read_fraction(p, {"vec": 4, "block": 128}) == 0.0
    assert bench.alg_bytes_per_node("f16", p, {"vec": 4, "block": 128}) == 36


@pytest.mark.parametrize("nx,launch,shape", [(37, (4, 64), (40, 6)), (96, (4, 128), (96, 5)),
                                             (160, (4, 256), (160, 6)), (130, (1, 64), (64, 1)),
                                             (3, (4, 64), (4, 64))])
def test_mask_fraction_3d_rows(bench, nx, launch, shape):
    """A 3-D mask is tiled as its nz ny lattice rows (row = z ny + y), a narrow
    grid's tile holding as many whole rows of nx rounded up to vec as fit."""
    from paper_1901_08766_amd import inputs3
    p = inputs3.random_state_problem3(nx, 11, 6, seed=5, n_spheres=2)
    launch = {"vec": launch[0], "block": launch[1]}
    tw, tr = bench.tile_shape(p.nx, launch, d3q19=True)
    assert (tw, tr) == shape
    rows = p.mask.reshape(-1, p.nx)
    count = 0
    for r0 in range(0, rows.shape[0], tr):
        for i0 in range(0, p.nx, tw):
            tile = rows[r0:r0 + tr, i0:i0 + tw]
            if (tile > 0).any():
                count += tile.size
    assert bench.mask_read_fraction(p, launch) == pytest.approx(count / rows.size, abs=0, rel=1e-15)
    assert bench.alg_bytes_per_node3("f16", p, launch) == 76 + count / rows.size
