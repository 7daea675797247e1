"""The D3Q19 entry points on the CPU: liblbvp.so exports every function that
include/lbvp3.h declares, the struct layouts agree with the Python binding, and
host-side validation rejects bad parameters before any device call."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbvp3.h")


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(lbvp3_\w+)\s*\(", text)))


def test_header_declares_the_named_calls():
    names = declared_functions()
    for must in ("lbvp3_create", "lbvp3_set_mask", "lbvp3_step", "lbvp3_forces", "lbvp3_read_fields"):
        assert must in names


def test_library_exports_every_declared_symbol(lbvp3):
    out = subprocess.run(["nm", "-D", "--defined-only", lbvp3._base.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (lbvp3_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(lbvp3.SYMBOLS) == set(declared_functions())


@pytest.mark.parametrize("name", ["lbvp3_params", "lbvp3_body"])
def test_struct_layouts_match_header(lbvp3, name):
    mirror = getattr(lbvp3, name)
    fields = [f[0] for f in mirror._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "lbvp3.h"', "int main(void) {",
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


def _good(lbvp3):
    p = lbvp3.lbvp3_params()
    p.nx, p.ny, p.nz = 40, 20, 10
    p.tau_plus, p.magic_lambda, p.eta, p.rho0 = 0.8, 0.25, 1e-4, 1.0
    p.rho_in = 1.0
    p.storage = 1
    p.force_every = 1
    return p


def test_host_validation(lbvp3):
    L = lbvp3._L
    p = _good(lbvp3)
    assert L.lbvp3_footprint_bytes(C.byref(p)) > 19 * 2 * 4 * 40 * 20 * 10
    out = C.c_void_p()
    bad_values = [("nz", 2), ("nx", 2), ("tau_plus", 0.5), ("magic_lambda", 0.0), ("eta", -1.0), ("rho0", 0.0),
                  ("storage", 7), ("force_every", -1), ("force_capacity", -2), ("max_bodies", 256), ("flags", 1),
                  ("bc_west", 1), ("bc_east", 5), ("rho_in", float("nan"))]
    for field, value in bad_values:
        q = lbvp3.lbvp3_params.from_buffer_copy(p)
        setattr(q, field, value)
        if field == "bc_west":        # exactly one periodic x side
            q.bc_east = 0
        assert L.lbvp3_footprint_bytes(C.byref(q)) == 0, field
        assert L.lbvp3_create(C.byref(q), None, C.byref(out)) == lbvp3.E_ARG, field
        assert lbvp3.lbvp3_last_error(None)
    q = lbvp3.lbvp3_params.from_buffer_copy(p)
    q.body_force[2] = float("inf")
    assert L.lbvp3_create(C.byref(q), None, C.byref(out)) == lbvp3.E_ARG
    assert L.lbvp3_step_count(None) == -1
    for fn in ("lbvp3_synchronize", "lbvp3_destroy"):
        assert getattr(L, fn)(None) == lbvp3.E_ARG
