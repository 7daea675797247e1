"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and runs the oracle pin tests against that build: every mutant must
make them fail. The real oracle is untouched.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbvp_ref.c")

MUTANTS = [
    ("guo factor applied twice", "(1.0 - 1.0 / (2.0 * tau_s)) * Fs",
     "(1.0 - 1.0 / (2.0 * tau_s)) * (1.0 - 1.0 / (2.0 * tau_s)) * Fs"),
    ("antisymmetric forcing factor dropped", "(1.0 - 1.0 / (2.0 * tau_a)) * Fa;", "Fa;"),
    ("rotation sign", "*UOx = B[2] - B[4] * (y - cy);", "*UOx = B[2] + B[4] * (y - cy);"),
    ("opposite map mirrored", "{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 6, 5}"),
    ("body-force half step dropped", "(jx + 0.5 * fbx)", "(jx)"),
    ("equilibrium at u*", "lbvp_ref_feq(rho, ux, uy, feq);", "lbvp_ref_feq(rho, usx, usy, feq);"),
    ("outflow from wrong column", "si = si < 0 ? 0 : nx - 1;", "si = si < 0 ? 0 : nx - 2;"),
    ("outflow from unshifted row", "si = si < 0 ? 0 : nx - 1;", "si = si < 0 ? 0 : nx - 1; sj = j;"),
    ("inflow at rho0", "return feq_one(a, c->p.rho_in,", "return feq_one(a, c->p.rho0,"),
    ("VP force missing factor 2", "out[2] = 2.0 * rho * c * (UOx - usx)", "out[2] = rho * c * (UOx - usx)"),
    ("force sign", "rf[2 * (b - 1)] -= fl[3];", "rf[2 * (b - 1)] += fl[3];"),
    ("tau_minus without 1/2", "return 0.5 + magic_lambda / (tau_plus - 0.5);",
     "return magic_lambda / (tau_plus - 0.5);"),
    ("equilibrium second-order term", "(eu * eu - CS2 * uu) / (2.0 * CS2 * CS2)",
     "(eu * eu - CS2 * uu) / (2.0 * CS2)"),
    ("lattice vector e6", "{0, 0, 1, 0, -1, 1, 1, -1, -1}", "{0, 0, 1, 0, -1, 1, -1, -1, 1}"),
    ("antisymmetric split sign", "fa = 0.5 * (f[a] - f[b]);", "fa = 0.5 * (f[a] + f[b]);"),
    ("guo velocity sign", "(EX[a] - ux) / CS2", "(EX[a] + ux) / CS2"),
    ("y not periodic", "sj = (sj % ny + ny) % ny;", "sj = sj < 0 ? 0 : (sj >= ny ? ny - 1 : sj);"),
    ("correction with eta not 2 eta", "out[0] = c * (UOx - usx) / (2.0 * eta + c);",
     "out[0] = c * (UOx - usx) / (eta + c);"),
    ("mass not summed over all rows", "for (int j = 0; j < ny; ++j) m += c->row_mass[j];",
     "for (int j = 1; j < ny; ++j) m += c->row_mass[j];"),
    ("moving body turned the wrong way", "const double xr = cs * dx + sn * dy + B[0];",
     "const double xr = cs * dx - sn * dy + B[0];"),
    ("moving body not translated", "*cx = B[0] + B[2] * t;", "*cx = B[0];"),
    ("moving mask one step behind", "const double t = (double)(c->step + 1);", "const double t = (double)(c->step);"),
    ("moving mask rounded down", "const double ir = floor(xr + 0.5), jr = floor(yr + 0.5);",
     "const double ir = floor(xr), jr = floor(yr);"),
    ("sampled step one time level behind",
     "node_update(c, g, xs[k], ys[k], (double)(c->step + 1), gout + Q * k, fl);",
     "node_update(c, g, xs[k], ys[k], (double)(c->step), gout + Q * k, fl);"),
    ("sampled step fields at the wrong stride", "fields[5 * k + q] = fl[q];", "fields[4 * k + q] = fl[q];"),
]


def _run_mutant(case, tmpdir):
    name, old, new = case
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    mutated = src.replace(old, new, 1)
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    c_path = os.path.join(tmpdir, f"{tag}.c")
    so_path = os.path.join(tmpdir, f"{tag}.so")
    with open(c_path, "w") as f:
        f.write(mutated)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", so_path, c_path, "-lm"], check=True)
    env = dict(os.environ, LBVP_REF_LIB=so_path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow",
                        os.path.join(ROOT, "tests", "test_oracle_node.py"),
                        os.path.join(ROOT, "tests", "test_oracle_grid.py"),
                        os.path.join(ROOT, "tests", "test_oracle_moving.py"),
                        os.path.join(ROOT, "tests", "test_oracle_step_nodes.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


@pytest.mark.slow
def test_pins_catch_planted_mistakes():
    with tempfile.TemporaryDirectory() as tmpdir:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda c: _run_mutant(c, tmpdir), MUTANTS))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, f"mutants not caught by the pins: {survived}"
