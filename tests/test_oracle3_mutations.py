"""The D3Q19 oracle's pins must catch plausible mistakes in it.

Each case plants one mistake in a copy of the oracle's C source (on the CPU),
builds it, and runs the D3Q19 oracle pin tests against that build: every mutant
must make them fail. The real oracle is untouched.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbvp3_ref.c")

MUTANTS = [
    ("edge vector z component", "1, -1, -1, 1, 1, -1, -1, 1};", "1, -1, -1, 1, 1, -1, 1, -1};"),
    ("edge weight", "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};",
     "1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0};"),
    ("opposite map", "13, 16, 15, 18, 17};", "13, 15, 16, 18, 17};"),
    ("rotation sign", "UO[2] = B[5] + (B[6] * r[1] - B[7] * r[0]);", "UO[2] = B[5] - (B[6] * r[1] - B[7] * r[0]);"),
    ("cross product component", "UO[1] = B[4] + (B[8] * r[0] - B[6] * r[2]);",
     "UO[1] = B[4] + (B[8] * r[1] - B[6] * r[2]);"),
    ("body offset along z taken from x", "double r[3] = {x - B[0], y - B[1], z - B[2]};",
     "double r[3] = {x - B[0], y - B[1], x - B[2]};"),
    ("z not periodic", "int sk = ((k - EZ3[a]) % nz + nz) % nz;",
     "int sk = k - EZ3[a] < 0 ? 0 : (k - EZ3[a] >= nz ? nz - 1 : k - EZ3[a]);"),
    ("z streamed the wrong way", "int sk = ((k - EZ3[a]) % nz + nz) % nz;", "int sk = ((k + EZ3[a]) % nz + nz) % nz;"),
    ("y pulled from the same row", "int sj = ((j - EY3[a]) % ny + ny) % ny;", "int sj = j;"),
    ("antisymmetric forcing factor dropped", "(1.0 - 1.0 / (2.0 * tau_a)) * Fa;", "Fa;"),
    ("antisymmetric split sign", "fa = 0.5 * (f[a] - f[b]);", "fa = 0.5 * (f[a] + f[b]);"),
    ("body-force half step dropped", "(j[d] + 0.5 * fb[d])", "(j[d])"),
    ("VP force missing factor 2", "fvp[d] = 2.0 * rho * c", "fvp[d] = rho * c"),
    ("correction with eta not 2 eta", "double du = c * (UO[d] - us) / (2.0 * eta + c);",
     "double du = c * (UO[d] - us) / (eta + c);"),
    ("equilibrium second-order term", "(eu * eu - CS2 * uu) / (2.0 * CS2 * CS2)", "(eu * eu - CS2 * uu) / (2.0 * CS2)"),
    ("guo velocity sign", "((e[d] - u[d]) / CS2", "((e[d] + u[d]) / CS2"),
    ("force sign", "pf[3 * (b - 1) + d] -= fl[4 + d];", "pf[3 * (b - 1) + d] += fl[4 + d];"),
    ("force summed over one plane", "out[q] += c->plane_force[(int64_t)3 * nb * k + q];", "out[q] += c->plane_force[q];"),
    ("mass not summed over all planes", "for (int k = 0; k < nz; ++k) m += c->plane_mass[k];",
     "for (int k = 1; k < nz; ++k) m += c->plane_mass[k];"),
    ("reported velocity before the correction", "fields[1 + d] = u[d];", "fields[1 + d] = u[d] - c * 0.5 * fvp[d] / fields[0];"),
    ("outflow from wrong column", "si = si < 0 ? 0 : nx - 1;", "si = si < 0 ? 0 : nx - 2;"),
    ("inflow at rho0", "return feq3_one(a, c->p.rho_in, c->p.u_in);", "return feq3_one(a, c->p.rho0, c->p.u_in);"),
    ("sampled step in the first plane", "node3_update(c, g, xs[k], ys[k], zs[k], gout + Q3 * k, fl);",
     "node3_update(c, g, xs[k], ys[k], 0, gout + Q3 * k, fl);"),
    ("sampled step with x and y swapped", "node3_update(c, g, xs[k], ys[k], zs[k], gout + Q3 * k, fl);",
     "node3_update(c, g, ys[k] % c->p.nx, xs[k] % c->p.ny, zs[k], gout + Q3 * k, fl);"),
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
    env = dict(os.environ, LBVP3_REF_LIB=so_path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow", os.path.join(ROOT, "tests", "test_oracle3.py"),
                        os.path.join(ROOT, "tests", "test_oracle_step_nodes.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


@pytest.mark.slow
def test_d3q19_pins_catch_planted_mistakes():
    with tempfile.TemporaryDirectory() as tmpdir:
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda c: _run_mutant(c, tmpdir), MUTANTS))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, f"mutants not caught by the pins: {survived}"
