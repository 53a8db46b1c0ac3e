"""Write film_dp45.txt and film_dp45_capped.txt: the float64 oracle's
adaptive Dormand-Prince runs of the 256 x 64 x 1 film (3.9 x 3.9 x 3 nm
cells, m0 tilted 10 deg from +x in the plane, applied field (-25, 4, 0) mT
from t = 0) to 1 ns, rtol = atol = 1e-5, dt0 = 1e-14 s, stopped at the output
times 0.1, 0.2, ..., 1.0 ns (each segment continues from the step the
controller proposed) (Sec. 5.3).  Each file holds the film average <m> and m
at 64 sampled nodes (seed 7) at every output time and every accepted step
(t, dt).

film_dp45.txt is the run as configured: the GPU's own adaptive run is
compared with it.  film_dp45_capped.txt caps the steps at 4e-13 s, inside the
stability region of the film's exchange modes: the uncapped controller first
takes steps outside it (the smooth error allows them) and then holds the
modes' rounding noise at the tolerance scale, so a float32 run forced onto
those steps amplifies its own noise, about 1e9 times the float64 one, instead
of following the method.  The GPU is made to take the capped run's steps.
Calls only the oracle and the input generator:

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
T_OUT = [0.1e-9 * (i + 1) for i in range(10)]


def sample_nodes(node_shape, count=64, seed=7):
    """Flat node indices (C order over (N3+1, N2+1, N1+1)), sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(node_shape)), size=count, replace=False))


def run(out, dt_max):
    p = synth.film()
    mesh, mat, m = to_oracle(p)
    idx = sample_nodes(mesh.node_shape)
    t, dt = 0.0, 1e-14
    rows, steps, rejected = [], [], 0
    t0 = time.perf_counter()
    for te in T_OUT:
        m, log, dt = oracle.dp45_solve(mesh, mat, m, t, te, dt, rtol=1e-5, atol=1e-5, dt_max=dt_max,
                                       return_dt=True)
        steps += [(a, b) for a, b, ok in log if ok]
        rejected += sum(1 for x in log if not x[2])
        t = te
        rows.append((te, m.mean(axis=(1, 2, 3)), m.reshape(3, -1)[:, idx]))
        print("%s t = %.2e s: %d accepted, %d rejected, <m> = %s (%.0f s)"
              % (os.path.basename(out), te, len(steps), rejected, rows[-1][1], time.perf_counter() - t0),
              flush=True)
    lines = ["# film 256x64x1 (synth.film), DP45 rtol = atol = 1e-5, dt0 = 1e-14 s, dt_max = %r s, "
             "float64 oracle;" % dt_max,
             "# written by tests/golden/make_film_dp45.py",
             "accepted %d rejected %d" % (len(steps), rejected),
             "nodes " + " ".join(str(int(i)) for i in idx),
             "# mean t_s mx my mz; then m at the sampled nodes (components 0, 1, 2)"]
    for te, mm, ms in rows:
        lines.append("mean %r %r %r %r" % (te, float(mm[0]), float(mm[1]), float(mm[2])))
        for c in range(3):
            lines.append("m%d %r " % (c, te) + " ".join(repr(float(v)) for v in ms[c]))
    lines.append("# step t_s dt_s (accepted steps, in order)")
    for a, b in steps:
        lines.append("step %r %r" % (a, b))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    from multiprocessing import Pool

    with Pool(2) as pool:
        pool.starmap(run, [(os.path.join(HERE, "film_dp45.txt"), np.inf),
                           (os.path.join(HERE, "film_dp45_capped.txt"), 4e-13)])


if __name__ == "__main__":
    main()
