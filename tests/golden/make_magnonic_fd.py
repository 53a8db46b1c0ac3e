"""Write magnonic_fd.txt: float64 central differences of the magnonic-strip
objective with respect to the per-cell applied-field map, for the full
256 x 128 x 1 strip over 4000 RK4 steps (Sec. 4: the gradient the adjoint
must reproduce), and, with --adjoint, the oracle's own discrete-adjoint
gradient at the same cells.  Calls only the oracle and the input generator:

    python tests/golden/make_magnonic_fd.py [--workers 6] [--adjoint] [--resume LOG]
                                            [--adjoint-from FILE]

--resume takes the progress lines ("run k/33: L = ...") an interrupted run
of this script printed and recomputes only the runs missing there;
--adjoint-from reuses the oracle-adjoint column of an earlier output.

Objective: L = -(1/K) sum_{k=1..K} mean over the output region's nodes (both
node layers) of m_z(t_k)^2, K = 4000, dt = 5e-14 s; the output region is the
nodes of cells 192 <= x < 208, 56 <= y < 72.  The 16 cells (one field
component each) are drawn from seed 105 away from the absorbing edges.
Each difference takes two float64 forward runs of 4000 steps (~15 min each
on one core); 32 runs are spread over worker processes.
"""
import argparse
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
from helpers import to_oracle  # noqa: E402
from oracle.adjoint import region_mz2_loss, rk4_gradient  # noqa: E402
from oracle.field import ALL_TERMS  # noqa: E402
from paper_2411_11725_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "magnonic_fd.txt")
NSTEPS = 4000
DT = 5e-14
H_FD = 1e-6 / (4e-7 * np.pi)      # 1e-3 mT (1e-6 T) in A/m
REGION = (slice(None), slice(56, 72), slice(192, 208))


def fd_cells():
    """16 (component, z, y, x) cells, seed 105, 16 <= x < 240, 16 <= y < 112."""
    rng = np.random.default_rng(105)
    out = []
    while len(out) < 16:
        c = (int(rng.integers(3)), 0, int(rng.integers(16, 112)), int(rng.integers(16, 240)))
        if c not in out:
            out.append(c)
    return out


def _problem():
    p = synth.magnonic()
    mesh, mat, m0 = to_oracle(p)
    region = np.zeros(mesh.node_shape, dtype=bool)
    region[REGION] = True
    return mesh, mat, m0, region


def objective(delta):
    """L with the field map theta = 0 except delta = (j, z, y, x, value)."""
    mesh, mat, m0, region = _problem()
    if delta is not None:
        j, z, y, x, v = delta
        hc = np.array(mat.h_cell)
        hc[j, z, y, x] += v
        mat = oracle.Material(**{**mat.__dict__, "h_cell": hc})
    loss, _ = region_mz2_loss(mesh, region, NSTEPS)
    m = m0.copy()
    tot = 0.0
    for k in range(NSTEPS):
        m = oracle.rk4_step(mesh, mat, m, k * DT, DT)
        tot += loss(m)
    return tot


def adjoint_gradient():
    mesh, mat, m0, region = _problem()
    _, dloss = region_mz2_loss(mesh, region, NSTEPS)
    _, dth, _ = rk4_gradient(mesh, mat, m0, DT, NSTEPS, dloss, ALL_TERMS)
    return dth


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--adjoint", action="store_true")
    ap.add_argument("--resume", help="progress lines of an interrupted run")
    ap.add_argument("--adjoint-from", help="an earlier output of this script whose oracle-adjoint column "
                                          "(independent of h) is reused instead of recomputed")
    args = ap.parse_args()
    from multiprocessing import Pool

    cells = fd_cells()
    jobs = [None] + [(j, z, y, x, s * H_FD) for (j, z, y, x) in cells for s in (1.0, -1.0)]
    vals = [None] * len(jobs)
    if args.resume:
        for line in open(args.resume):
            if line.startswith("run ") and "/%d: L = " % len(jobs) in line:
                k = int(line.split()[1].split("/")[0])
                vals[k - 1] = float(line.split("=")[1])
    todo = [k for k in range(len(jobs)) if vals[k] is None]
    with Pool(args.workers) as pool:
        adj = pool.apply_async(adjoint_gradient) if args.adjoint else None
        for k, v in zip(todo, pool.imap(objective, [jobs[k] for k in todo])):
            vals[k] = v
            print("run %d/%d: L = %.17e" % (k + 1, len(jobs), v), flush=True)
        dth = adj.get() if adj is not None else None
    if args.adjoint_from:
        dth = np.zeros((3, 1, 128, 256))
        got = 0
        for line in open(args.adjoint_from):
            w = line.split()
            if len(w) == 8 and not w[0].startswith("#"):
                dth[int(w[0]), int(w[1]), int(w[2]), int(w[3])] = float(w[7])
                got += 1
            elif w and w[0] == "adjoint_max_abs":
                adj_max = float(w[1])
        assert got == len(cells)
    L0 = vals[0]
    lines = ["# magnonic strip 256x128x1 (synth.magnonic), RK4 dt 5e-14 s x 4000, field map theta = 0;",
             "# L = -(1/4000) sum_k mean over nodes [:, 56:72, 192:208] of m_z(t_k)^2;",
             "# central differences with h = 1e-3 mT = %.10e A/m (written by tests/golden/make_magnonic_fd.py)"
             % H_FD,
             "L0 %.17e" % L0,
             "# component z y x  dL/dtheta_fd  L(+h)  L(-h)  [dL/dtheta oracle adjoint]"]
    for i, (j, z, y, x) in enumerate(cells):
        lp, lm = vals[1 + 2 * i], vals[2 + 2 * i]
        fd = (lp - lm) / (2.0 * H_FD)
        row = "%d %d %3d %3d % .17e % .17e % .17e" % (j, z, y, x, fd, lp, lm)
        if dth is not None:
            row += " % .17e" % dth[j, z, y, x]
        lines.append(row)
    if dth is not None:
        lines.append("adjoint_max_abs %.17e" % (adj_max if args.adjoint_from else np.abs(dth).max()))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
