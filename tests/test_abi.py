"""The C-ABI library on the CPU: it loads, exports every entry point that
include/lbvp.h declares, its struct layouts agree with the Python binding, and
host-side validation rejects bad parameters before any GPU work. No compute call
is made here (there may be no GPU)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbvp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbvp_\w+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = declared_functions()
    for must in ("lbvp_create", "lbvp_set_mask", "lbvp_step", "lbvp_forces", "lbvp_read_fields"):
        assert must in names


def test_library_exports_every_declared_symbol(lbvp):
    out = subprocess.run(["nm", "-D", "--defined-only", lbvp.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (lbvp_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(lbvp.SYMBOLS) <= exported
    for name in declared_functions():
        getattr(lbvp.lib(), name)


@pytest.mark.parametrize("name", ["lbvp_params", "lbvp_body", "lbvp_tune_row", "lbvp_pool_config",
                                  "lbvp_pool_stats"])
def test_struct_layouts_match_header(lbvp, name):
    """Compile a C probe of the header with gcc and compare sizeof/offsetof with
    the ctypes mirrors used by the binding."""
    mirror = getattr(lbvp, name)
    fields = [f[0] for f in mirror._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbvp.h"', "int main(void) {",
           f'printf("%zu\\n", sizeof({name}));']
    src += [f'printf("%zu\\n", offsetof({name}, {f}));' for f in fields]
    src += ["return 0; }"]
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write("\n".join(src))
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == C.sizeof(mirror)
    for f, off in zip(fields, vals[1:]):
        assert getattr(mirror, f).offset == off, f
    assert len(vals) == len(fields) + 1


def test_pool_and_tuner_reject_bad_arguments_on_the_host(lbvp):
    """Argument checks that return before any device call."""
    L = lbvp.lib()
    cfg = lbvp.lbvp_pool_config()
    cfg.cap_bytes, cfg.max_slots, cfg.storage = 1 << 30, 4, 1
    out = C.c_void_p()
    assert L.lbvp_pool_create(C.byref(cfg), None, C.byref(out)) == lbvp.E_ARG      # null stream
    fake_stream = C.c_void_p(1)                                                     # never used: checks come first
    for field, value in [("max_slots", 0), ("storage", 9), ("layout_flags", 4), ("block", 32),
                         ("vec", 3), ("max_in_flight", -1), ("cap_bytes", 0)]:
        bad = lbvp.lbvp_pool_config.from_buffer_copy(cfg)
        setattr(bad, field, value)
        assert L.lbvp_pool_create(C.byref(bad), fake_stream, C.byref(out)) == lbvp.E_ARG, field
        assert lbvp.lbvp_pool_last_error(None)
    aa16 = lbvp.lbvp_pool_config.from_buffer_copy(cfg)
    aa16.storage, aa16.layout_flags, aa16.vec = 2, lbvp.LAYOUT_AA, 8   # 2-byte AA runs one node per thread
    assert L.lbvp_pool_create(C.byref(aa16), fake_stream, C.byref(out)) == lbvp.E_ARG
    rows = (lbvp.lbvp_tune_row * 4)()
    n, best = C.c_int32(), C.c_int32()
    assert L.lbvp_tune(None, 0, 10, 0, rows, 4, C.byref(n), C.byref(best)) == lbvp.E_ARG
    assert lbvp.lbvp_tune_last_error()
    assert L.lbvp_pool_admit(None, None, None, 0, None, None, None, None, 1, None) == lbvp.E_ARG
    assert L.lbvp_pool_destroy(None) == lbvp.OK


def _params(lbvp, **kw):
    from paper_1901_08766_amd import inputs
    p = lbvp.params_for(inputs.cylinder(nx=64, ny=32, d=8, cx=16, cy=16, noise=False))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [("nx", 2), ("ny", 0), ("tau_plus", 0.5), ("magic_lambda", 0.0),
                                         ("eta", -1.0), ("storage", 7), ("bc_north", 1), ("bc_west", 0),
                                         ("force_every", -1), ("max_bodies", 256), ("flags", 0x80),
                                         ("rho0", float("nan"))])
def test_create_rejects_invalid_parameters(lbvp, field, value):
    p = _params(lbvp, **{field: value})
    assert lbvp.lbvp_footprint_bytes(p) == 0
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_create(p)
    assert e.value.status == lbvp.E_ARG
    assert lbvp.lbvp_last_error(None)


def test_footprint_scales_with_storage(lbvp):
    sizes = {st: lbvp.lbvp_footprint_bytes(_params(lbvp, storage=code)) for st, code in lbvp.STORAGE.items()}
    assert all(v > 0 for v in sizes.values())
    assert sizes["f64"] > sizes["f32"] > sizes["f16"] == sizes["bf16"]


def test_create_rejects_small_borrowed_memory(lbvp):
    p = _params(lbvp)
    need = lbvp.lbvp_footprint_bytes(p)
    with pytest.raises(lbvp.LbvpError) as e:
        lbvp.lbvp_create(p, None, 256, need - 1)   # never dereferenced: the size check fails first
    assert e.value.status == lbvp.E_NOMEM


def test_device_copy_rejects_misaligned_arguments(lbvp):
    L = lbvp.lib()
    assert L.lbvp_device_copy(C.c_void_p(16), C.c_void_p(32), 17, None) == lbvp.E_ARG
    assert L.lbvp_device_copy(C.c_void_p(8), C.c_void_p(32), 16, None) == lbvp.E_ARG
    assert L.lbvp_device_copy(None, C.c_void_p(32), 16, None) == lbvp.E_ARG
    assert L.lbvp_device_copy(C.c_void_p(16), C.c_void_p(32), 0, None) == lbvp.OK


def test_moving_bodies_limit(lbvp):
    p = _params(lbvp, flags=lbvp.MOVING_BODIES, max_bodies=9)
    out = C.c_void_p()
    assert lbvp.lib().lbvp_create(C.byref(p), None, None, 0, C.byref(out)) == lbvp.E_ARG
    assert "moving" in lbvp.lbvp_last_error(None)


def test_neighbor_sides_validation(lbvp):
    """A cut side needs the two-lattice layout and a fixed mask; with one
    periodic x side it is rejected like any other mixed pair; the exchange
    rejects NULL links before any device call."""
    nb = lbvp.BC["neighbor"]
    assert lbvp.lbvp_footprint_bytes(_params(lbvp, bc_west=nb, bc_east=nb)) > 0
    assert lbvp.lbvp_footprint_bytes(_params(lbvp, bc_west=1, bc_east=nb)) > 0
    for kw in ({"bc_west": nb, "bc_east": nb, "flags": lbvp.LAYOUT_AA},
               {"bc_west": nb, "bc_east": 2, "flags": lbvp.MOVING_BODIES},
               {"bc_west": nb, "bc_east": 0}, {"bc_west": 4, "bc_east": nb}):
        assert lbvp.lbvp_footprint_bytes(_params(lbvp, **kw)) == 0, kw
    L = lbvp.lib()
    assert L.lbvp_halo_exchange(None, None, 1) == lbvp.E_ARG
    arr = (C.c_void_p * 1)(None)
    assert L.lbvp_halo_exchange(arr, arr, 1) == lbvp.E_ARG
    assert L.lbvp_halo_exchange(arr, arr, 0) == lbvp.E_ARG
