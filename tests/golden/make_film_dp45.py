"""Write film_dp45.txt: the float64 oracle's adaptive Dormand-Prince run of
the 256 x 64 x 1 film (3.9 x 3.9 x 3 nm cells, m0 tilted 10 deg from +x in
the plane, applied field (-25, 4, 0) mT from t = 0) to 1 ns, rtol = atol =
1e-5, dt0 = 1e-14 s, stopped at the output times 0.1, 0.2, ..., 1.0 ns (each
segment continues from the step the controller proposed).  Stores the film
average <m> at every output time and every accepted step (t, dt), so that
the GPU can be run independently to the same output times and made to take
the oracle's accepted steps (Sec. 5.3).  Calls only the oracle and the input
generator:

    python tests/golden/make_film_dp45.py
"""
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
from helpers import to_oracle  # noqa: E402
from paper_2411_11725_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "film_dp45.txt")
T_OUT = [0.1e-9 * (i + 1) for i in range(10)]


def main():
    p = synth.film()
    mesh, mat, m = to_oracle(p)
    t, dt = 0.0, 1e-14
    means, steps, rejected = [], [], 0
    t0 = time.perf_counter()
    for te in T_OUT:
        m, log, dt = oracle.dp45_solve(mesh, mat, m, t, te, dt, rtol=1e-5, atol=1e-5, return_dt=True)
        steps += [(a, b) for a, b, ok in log if ok]
        rejected += sum(1 for x in log if not x[2])
        t = te
        means.append(m.mean(axis=(1, 2, 3)))
        print("t = %.2e s: %d accepted, %d rejected, <m> = %s (%.0f s)"
              % (te, len(steps), rejected, means[-1], time.perf_counter() - t0), flush=True)
    lines = ["# film 256x64x1 (synth.film), DP45 rtol = atol = 1e-5, dt0 = 1e-14 s, float64 oracle;",
             "# written by tests/golden/make_film_dp45.py",
             "accepted %d rejected %d" % (len(steps), rejected),
             "# mean t_s mx my mz"]
    for te, mm in zip(T_OUT, means):
        lines.append("mean %r %r %r %r" % (te, float(mm[0]), float(mm[1]), float(mm[2])))
    lines.append("# step t_s dt_s (accepted steps, in order)")
    for a, b in steps:
        lines.append("step %r %r" % (a, b))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
