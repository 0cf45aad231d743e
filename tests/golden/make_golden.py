"""Write the stored expected values of the parity tests.

Calls only the oracle (and the seeded input generator):
  fstar_c0.txt  - exact LP optimum F* of all 9 plans of the small case
  fstar_c1.txt  - exact LP optimum F* of sampled plans of the medium case
Run from the repository root:  python tests/golden/make_golden.py [c0|c1 ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import cases                      # noqa: E402
from oracle import lp as olp                 # noqa: E402
from oracle.simplex import solve_plan, kkt_residuals   # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLES = {0: list(range(9)), 1: [0, 8, 40, 72, 80]}


def write(config):
    case = cases.make_case(config)
    w = cases.config_weights(config)
    lp = olp.assemble(case, w)
    lines = [f"# Exact optimum F* = -p* of the planning LP (App. A dual solved by the oracle's",
             f"# dense bounded simplex, KKT-certified) for the synthetic case {case.name},",
             f"# seed {case.seed}; weights from the {cases.CONFIG_PLANS[config]}x"
             f"{cases.CONFIG_PLANS[config]} slider grid.  Written by make_golden.py.",
             "# plan w_T w_R w_LD w_BOT F* kkt_primal kkt_dual"]
    for j in SAMPLES[config]:
        t0 = time.time()
        res = solve_plan(lp, j)
        assert res.status == "optimal", res.status
        kkt = kkt_residuals(lp.A, lp.b[:, j], lp.c, lp.u[:, j], res.x, res.lam)
        lines.append(f"{j} {w[j, 0]:.17g} {w[j, 1]:.17g} {w[j, 2]:.17g} {w[j, 3]:.17g} "
                     f"{-res.objective:.17g} {kkt['primal']:.2e} {kkt['dual']:.2e}")
        print(f"config {config} plan {j}: F* = {-res.objective:.10g} ({time.time() - t0:.1f} s, "
              f"{res.iterations} pivots)", flush=True)
    with open(os.path.join(HERE, f"fstar_c{config}.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


def read(config):
    rows = [l.split() for l in open(os.path.join(HERE, f"fstar_c{config}.txt"))
            if l.strip() and not l.startswith("#")]
    return {int(r[0]): float(r[5]) for r in rows}


if __name__ == "__main__":
    for arg in sys.argv[1:] or ["c0", "c1"]:
        write(int(arg[1:]))
