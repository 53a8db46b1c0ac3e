"""Write depinning_fields.txt: the float64 oracle's depinning fields of the
two-phase chains (oracle.depinning.discrete_depinning_field, bisection to a
relative bracket of 1e-3) and their closed-form continuum limit.  Calls only
the oracle and the input generator:

    python tests/golden/make_depinning.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from helpers import to_oracle  # noqa: E402
from oracle import depinning as dp  # noqa: E402
from paper_2411_11725_amd import synth  # noqa: E402

SPACINGS = (1e-9, 0.5e-9)


def main():
    lines = ["# case hx_m closed_form_T oracle_lo_T oracle_hi_T  (mu0 H_p; chain of synth.two_phase_chain,",
             "# 60 nm soft + 30 nm hard, cubic cells; written by tests/golden/make_depinning.py)"]
    for hx in SPACINGS:
        for case in synth.DEPIN_CASES:
            p = synth.two_phase_chain(case, hx=hx)
            mesh, mat, m0 = to_oracle(p)
            bc = dp.closed_form_field(*synth.depinning_phases(case))
            lo, hi = dp.discrete_depinning_field(mesh, mat, m0, p["n_soft"], 0.5 * bc, 1.5 * bc, rel_tol=1e-3)
            lines.append("%-7s %.3e %.6f %.6f %.6f" % (case, hx, bc, lo, hi))
            print(lines[-1], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "depinning_fields.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
