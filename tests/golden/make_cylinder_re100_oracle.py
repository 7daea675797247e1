"""Write the oracle's shedding statistics for the single-cylinder case
(1024 x 512, D = 40 at (256, 256), U = 0.05, Re = 100, Lambda = 3/16,
eta = 1e-4, seeded noise 2, 200k steps; paper Sec. 3.2, Table high-Re).

Calls only the oracle and the shared input generators. The statistics use the
oracle-side post-processing over steps 100k-200k: mean drag coefficient, drag
and lift amplitudes ((max - min)/2) and the Strouhal number from upward zero
crossings of the lift coefficient. Run time is about an hour on 8 cores.

    python tests/golden/make_cylinder_re100_oracle.py [--steps N]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import diag, ref  # noqa: E402
from paper_1901_08766_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cylinder_re100_oracle.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200_000)
    ap.add_argument("--chunk", type=int, default=10_000)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    p = inputs.cylinder(steps=a.steps)
    s = ref.RefSolver(p)
    forces, mass = [], []
    t0 = time.time()
    done = 0
    while done < a.steps:
        n = min(a.chunk, a.steps - done)
        f, m = s.step(n, record=True)
        forces.append(f[:, 0, :])
        mass.append(m)
        done += n
        el = time.time() - t0
        print(f"step {done}/{a.steps}  {el:.0f}s  {p.nx * p.ny * done / el / 1e6:.1f} MLUPS  "
              f"Cd={2 * f[-1, 0, 0] / (p.u_ref ** 2 * p.l_ref):.4f}", flush=True)
    forces = np.concatenate(forces)
    mass = np.concatenate(mass)
    half = a.steps // 2
    summary = diag.shedding_summary(forces[half:], 1.0, p.u_ref, p.l_ref)
    samples = {str(k): [float(forces[k - 1, 0]), float(forces[k - 1, 1])]
               for k in (1, 10, 100, 1000, 10_000) if k <= a.steps}
    out = {
        "what": "oracle FP64 shedding statistics, single cylinder Re=100 (1024x512, D=40, U=0.05, "
                "Lambda=3/16, eta=1e-4, noise seed 2)",
        "steps": a.steps,
        "window": [half, a.steps],
        "summary": summary,
        "force_on_body_at_step": samples,
        "mass_first_last": [float(mass[0]), float(mass[-1])],
        "oracle_threads": ref.num_threads(),
        "seconds": time.time() - t0,
    }
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out["summary"]))


if __name__ == "__main__":
    main()
