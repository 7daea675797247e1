"""Vortex shedding behind a cylinder (Re = 100, Sec. 3.2, Table high-Re): the
FP32 GPU run against the FP64 oracle's 200k-step run stored in
tests/golden/cylinder_re100_oracle.json (written by make_cylinder_re100_oracle.py,
which calls only the oracle).

Pointwise fields decorrelate once shedding starts (round-off moves the phase),
so the comparison is statistical over steps 100k-200k: mean drag coefficient,
lift amplitude and Strouhal number within 0.5%. Before shedding the force
history is deterministic and is compared sample by sample."""
import json
import os

import numpy as np
import pytest

from oracle import diag
from paper_1901_08766_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cylinder_re100_oracle.json")


def test_shedding_statistics_match_oracle(lbvp):
    gold = json.load(open(GOLDEN))
    prob = inputs.cylinder(steps=gold["steps"])
    s = lbvp.Solver(prob, storage="f32", force_every=1, force_capacity=16384)
    print(f"cylinder {prob.nx}x{prob.ny} f32 launch={s.launch}: {gold['steps']} steps", flush=True)
    forces, mass = s.run(gold["steps"], chunk=16384)
    assert forces.shape == (gold["steps"], 1, 2) and np.all(np.isfinite(mass))
    for k, (fx, fy) in gold["force_on_body_at_step"].items():
        k = int(k)
        assert abs(forces[k - 1, 0, 0] - fx) <= 1e-4 * abs(fx), k
    lo, hi = gold["window"]
    got = diag.shedding_summary(forces[lo:hi, 0, :], 1.0, prob.u_ref, prob.l_ref)
    ref = gold["summary"]
    print("GPU", got, "\noracle", ref, flush=True)
    for key in ("cd_mean", "cl_amp", "st"):
        assert abs(got[key] - ref[key]) <= 5e-3 * abs(ref[key]), key
