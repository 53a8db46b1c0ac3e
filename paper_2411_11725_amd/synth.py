"""Seeded synthetic inputs (meshes, materials, initial magnetisations).

This module holds no arithmetic of the method: it only draws random numbers
and lays out parameter arrays.  Both the GPU path and its checker take their
inputs from here, rounded to float32 (the GPU's storage precision), so that
both start from bit-identical values.

Workloads (every value in SI; mT fields are converted with H = B / mu0):
  standard_cube   16 x 16 x 4 cells of 2 nm, Ms 8e5, A 1.3e-11, alpha 0.02,
                  random unit m0 per node (seed 101)
  film            256 x 64 x 1 cells of 3.9 x 3.9 x 3 nm, Ms 8e5, A 1.3e-11,
                  alpha 0.02, m0 tilted 10 deg from +x in-plane, field step
                  (-25, 4, 0) mT
  block           128 x 128 x 32 cells of 2 nm, Ms 1e6, A 1.5e-11, alpha 1,
                  Ku ~ U[0, 5e5] per cell, easy axes uniform on the sphere,
                  random unit m0 per node (seed 103)
  magnonic        256 x 128 x 1 cells of 4 x 4 x 5 nm, Ms 1.4e5, A 3.5e-12,
                  alpha 1e-3 ramped linearly to 0.5 over the outer 16 cells of
                  every in-plane edge, per-cell field map (init 0), 1 mT drive
                  along +y at 10 GHz on the cells 16 <= x < 20
  two_phase_chain a chain of cells along x (2 across), 60 nm of a soft phase then 30 nm
                  of a hard phase (A 1e-11, K 1e6, Ms 1e6; the soft phase
                  differs in the named ones of A 2.5e-12, K 1e5, Ms 1.5e6),
                  easy axis z, alpha 1, a wall in the soft phase
"""
import math

import numpy as np

MU0_SI = 4.0e-7 * math.pi  # only to convert mT inputs to A/m


def random_unit_vectors(count, rng):
    """Gaussian 3-vectors normalised to unit length, shape (3, count)."""
    v = rng.standard_normal((3, count))
    return v / np.linalg.norm(v, axis=0, keepdims=True)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def make_problem(n, h, Ms, A, alpha, gamma=2.211e5, m0="random", seed=0,
                 Ku=None, easy="random", h_uniform=(0.0, 0.0, 0.0),
                 h_cell=None, drive_mask=None, drive_amp=(0.0, 0.0, 0.0),
                 drive_freq=0.0, drive_phase=0.0, D=None):
    """Return a dict of float32 arrays describing one problem.

    Cell arrays have shape (N3, N2, N1), cell vectors (3, N3, N2, N1) and the
    nodal magnetisation (3, N3+1, N2+1, N1+1): C order, x fastest.
    Scalars Ms, A, alpha, Ku may be numbers (uniform) or cell arrays.
    """
    n1, n2, n3 = n
    cells = (n3, n2, n1)
    nodes = (n3 + 1, n2 + 1, n1 + 1)
    rng = np.random.default_rng(seed)

    def cellv(x):
        return _f32(np.broadcast_to(np.asarray(x, dtype=np.float64), cells))

    out = {"n": tuple(n), "h": tuple(float(v) for v in h), "gamma": float(gamma)}
    out["Ms"] = cellv(Ms)
    out["A"] = cellv(A)
    out["alpha"] = cellv(alpha)
    if isinstance(m0, str) and m0 == "random":
        m = random_unit_vectors(int(np.prod(nodes)), rng).reshape((3,) + nodes)
    else:
        m = np.broadcast_to(np.asarray(m0, dtype=np.float64).reshape(3, 1, 1, 1),
                            (3,) + nodes)
    out["m0"] = _f32(m)
    if Ku is not None:
        if isinstance(Ku, tuple) and Ku[0] == "uniform":
            out["Ku"] = _f32(rng.uniform(Ku[1], Ku[2], size=cells))
        else:
            out["Ku"] = cellv(Ku)
        if isinstance(easy, str) and easy == "random":
            out["easy"] = _f32(random_unit_vectors(int(np.prod(cells)), rng).reshape((3,) + cells))
        else:
            out["easy"] = _f32(np.broadcast_to(np.asarray(easy, dtype=np.float64).reshape(3, 1, 1, 1),
                                               (3,) + cells))
    else:
        out["Ku"] = None
        out["easy"] = None
    out["h_uniform"] = np.asarray(h_uniform, dtype=np.float32)
    out["h_cell"] = None if h_cell is None else _f32(h_cell)
    out["drive_mask"] = None if drive_mask is None else _f32(drive_mask)
    out["drive_amp"] = np.asarray(drive_amp, dtype=np.float32)
    out["drive_freq"] = float(drive_freq)
    out["drive_phase"] = float(drive_phase)
    out["D"] = None if D is None else cellv(D)
    return out


def standard_cube(seed=101):
    return make_problem((16, 16, 4), (2e-9, 2e-9, 2e-9), 8.0e5, 1.3e-11, 0.02,
                        seed=seed)


def film(seed=102, n=(256, 64, 1)):
    th = math.radians(10.0)
    return make_problem(n, (3.9e-9, 3.9e-9, 3e-9), 8.0e5, 1.3e-11, 0.02,
                        m0=(math.cos(th), math.sin(th), 0.0), seed=seed,
                        h_uniform=(-25e-3 / MU0_SI, 4e-3 / MU0_SI, 0.0))


def block(n=(128, 128, 32), seed=103, D=None):
    return make_problem(n, (2e-9, 2e-9, 2e-9), 1.0e6, 1.5e-11, 1.0, seed=seed,
                        Ku=("uniform", 0.0, 5e5), easy="random", D=D)


def magnonic(n=(256, 128, 1), seed=105):
    n1, n2, n3 = n
    ramp = 16
    x = np.arange(n1)
    y = np.arange(n2)
    # distance (in cells) to the nearest in-plane edge
    dx = np.minimum(x, n1 - 1 - x)[None, :]
    dy = np.minimum(y, n2 - 1 - y)[:, None]
    dist = np.minimum(dx, dy).astype(np.float64)
    frac = np.clip((ramp - dist) / ramp, 0.0, 1.0)
    alpha = 1e-3 + (0.5 - 1e-3) * frac
    alpha = np.broadcast_to(alpha, (n3, n2, n1))
    mask = np.zeros((n3, n2, n1))
    mask[:, :, 16:20] = 1.0
    return make_problem(n, (4e-9, 4e-9, 5e-9), 1.4e5, 3.5e-12, alpha,
                        m0=(1.0, 0.0, 0.0), seed=seed,
                        h_cell=np.zeros((3, n3, n2, n1)), drive_mask=mask,
                        drive_amp=(0.0, 1e-3 / MU0_SI, 0.0), drive_freq=10e9)


def as_film(p):
    """The same single-layer problem under the thin-film basis: one node layer
    (the lower one of m0), the cell arrays unchanged."""
    if p["n"][2] != 1:
        raise ValueError("the film basis takes one layer of cells")
    q = dict(p)
    q["basis"] = "film"
    q["m0"] = np.ascontiguousarray(p["m0"][:, :1])
    return q


def small_random(n, h=(2e-9, 2e-9, 2e-9), seed=7, anis=True, field=True,
                 hetero=True, ku_range=(0.0, 5e5), dmi=False, dmi_type="interfacial", cubic=False):
    """Small heterogeneous problem used by the parity tests: every term on,
    per-cell Ms, A, alpha, Ku ~ U[ku_range] (a negative Ku makes the cell
    easy-plane), easy axes and applied field; with dmi, a DMI constant
    D ~ U[-3e-3, 3e-3] J/m^2 per cell of the given kind ("interfacial" or
    "bulk"); with cubic, a cubic anisotropy Kc ~ U[-4e5, 4e5] J/m^3 and
    random orthonormal cubic axes (c1, c2) per cell."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    cells = (n3, n2, n1)
    Ms = rng.uniform(4e5, 1.2e6, size=cells) if hetero else 8e5
    A = rng.uniform(5e-12, 2e-11, size=cells) if hetero else 1.3e-11
    alpha = rng.uniform(0.01, 0.5, size=cells) if hetero else 0.1
    hc = rng.uniform(-5e4, 5e4, size=(3,) + cells) if field else None
    D = rng.uniform(-3e-3, 3e-3, size=cells) if dmi else None
    p = make_problem(n, h, Ms, A, alpha, seed=seed + 1,
                     Ku=("uniform",) + tuple(ku_range) if anis else None,
                     easy="random", h_uniform=(1e4, -2e4, 3e4) if field else (0, 0, 0),
                     h_cell=hc, D=D)
    p["dmi_type"] = dmi_type
    if cubic:
        nc = n1 * n2 * n3
        c1 = random_unit_vectors(nc, rng)
        r = random_unit_vectors(nc, rng)
        c2 = np.cross(c1, r, axis=0)
        c2 /= np.linalg.norm(c2, axis=0, keepdims=True)
        p["Kc"] = _f32(rng.uniform(-4e5, 4e5, size=cells))
        p["cubic"] = _f32(np.concatenate([c1, c2]).reshape((6,) + cells))
    return p


def serving_requests(count, seed=104, rate=200.0, nmin=32, nmax=512, nzmax=8, h=3e-9):
    """Poisson stream of solve requests: exponential inter-arrival gaps at
    `rate` per second; nx, ny rounded from log-uniform [nmin, nmax], nz uniform
    in 1..nzmax; cubic h cells; Ms ~ U[4e5, 1.2e6]; alpha log-uniform in
    [0.005, 0.5]; A = 1.3e-11; random unit m0 per node.  Returns a list of
    (arrival time in s, problem dict)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        if i:
            t += rng.exponential(1.0 / rate)
        nx = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        ny = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        nz = int(rng.integers(1, nzmax + 1))
        Ms = rng.uniform(4e5, 1.2e6)
        alpha = math.exp(rng.uniform(math.log(0.005), math.log(0.5)))
        p = make_problem((nx, ny, nz), (h, h, h), Ms, 1.3e-11, alpha,
                         seed=int(rng.integers(1 << 31)))
        out.append((t, p))
    return out


# two-phase depinning: phase 2 (hard) is the same in every case, phase 1
# (soft) takes the soft value of each parameter the case names
DEPIN_HARD = dict(A=1.0e-11, K=1.0e6, Ms=1.0e6)
DEPIN_SOFT = dict(A=2.5e-12, K=1.0e5, Ms=1.5e6)
DEPIN_CASES = ("A/K/Ms", "A/K", "A/Ms", "A", "K/Ms", "K")


def depinning_phases(case):
    """((A1, K1, Ms1), (A2, K2, Ms2)) of a two-phase case such as "A/K"."""
    names = case.split("/")
    if case not in DEPIN_CASES:
        raise ValueError("unknown two-phase case %r" % case)
    p1 = tuple(DEPIN_SOFT[k] if k in names else DEPIN_HARD[k] for k in ("A", "K", "Ms"))
    p2 = tuple(DEPIN_HARD[k] for k in ("A", "K", "Ms"))
    return p1, p2


def two_phase_chain(case, hx=1e-9, hyz=None, soft_len=60e-9, hard_len=30e-9):
    """N1 x 2 x 1 cells of hx x hyz x hyz along x (two across, the fewest
    the library takes; hyz defaults to hx): the soft phase, then the hard
    phase; easy axis +z in both, alpha 1, no applied field.  With cells much
    longer across than along the chain, a narrow wall lowers its energy by a
    checkerboard of its in-plane part across the section (a spurious mode of
    the under-resolved section), so the chains use cubic cells.  m0 is a
    wall in the plane x = 0 (m = (0, sin theta, cos theta)) from theta = pi
    at x = 0 to theta = 0, of width sqrt(A1/K1), centred two widths before
    the interface.  Extra key "n_soft": cells of the soft phase."""
    (A1, K1, M1), (A2, K2, M2) = depinning_phases(case)
    hyz = hx if hyz is None else hyz
    n1 = int(round(soft_len / hx))
    n2 = int(round(hard_len / hx))
    soft = np.arange(n1 + n2) < n1
    cells = (1, 2, n1 + n2)
    sel = lambda a, b: np.broadcast_to(np.where(soft, a, b), cells)
    w = math.sqrt(A1 / K1)
    x = np.arange(n1 + n2 + 1) * hx
    theta = 2.0 * np.arctan(np.exp(-(x - (n1 * hx - 2.0 * w)) / w))
    m = np.zeros((3, 2, 3, n1 + n2 + 1))
    m[1] = np.sin(theta)
    m[2] = np.cos(theta)
    p = make_problem((n1 + n2, 2, 1), (hx, hyz, hyz), sel(M1, M2), sel(A1, A2), 1.0, m0=(0.0, 0.0, 1.0),
                     Ku=sel(K1, K2), easy=(0.0, 0.0, 1.0))
    p["m0"] = _f32(m)
    p["n_soft"] = n1
    return p


def embed_in_vacuum(p, n_big, offset, seed=109):
    """The problem p placed at cell offset (o1, o2, o3) inside a mesh of n_big
    cells whose other cells are vacuum (Ms = 0, A = 0, Ku = 0, no field,
    alpha 0.1, easy axis z, D = 0).  Nodes touching the core keep p's m0;
    the rest get random unit vectors (seed), which the method must ignore."""
    n1, n2, n3 = p["n"]
    o1, o2, o3 = offset
    N1, N2, N3 = n_big
    if o1 + n1 > N1 or o2 + n2 > N2 or o3 + n3 > N3 or min(offset) < 0:
        raise ValueError("the core does not fit")
    cs = (slice(o3, o3 + n3), slice(o2, o2 + n2), slice(o1, o1 + n1))
    ns = (slice(o3, o3 + n3 + 1), slice(o2, o2 + n2 + 1), slice(o1, o1 + n1 + 1))
    big = (N3, N2, N1)

    def cell(a, fill):
        if a is None:
            return None
        a = np.asarray(a, dtype=np.float64)
        lead = a.shape[:-3]
        out = np.broadcast_to(np.asarray(fill, dtype=np.float64).reshape(lead + (1, 1, 1)) if lead else fill,
                              lead + big).copy()
        out[(Ellipsis,) + cs] = a
        return _f32(out)

    q = dict(p)
    q["n"] = tuple(n_big)
    q["Ms"] = cell(p["Ms"], 0.0)
    q["A"] = cell(p["A"], 0.0)
    q["alpha"] = cell(p["alpha"], 0.1)
    q["Ku"] = cell(p["Ku"], 0.0)
    q["easy"] = cell(p["easy"], (0.0, 0.0, 1.0))
    q["h_cell"] = cell(p["h_cell"], (0.0, 0.0, 0.0))
    q["drive_mask"] = cell(p["drive_mask"], 0.0)
    q["D"] = cell(p.get("D"), 0.0)
    rng = np.random.default_rng(seed)
    m = random_unit_vectors((N3 + 1) * (N2 + 1) * (N1 + 1), rng).reshape(3, N3 + 1, N2 + 1, N1 + 1)
    m[(slice(None),) + ns] = p["m0"]
    q["m0"] = _f32(m)
    return q


def wall_chain(hx=0.5e-9, length=60e-9, A=1e-11, K=1e6, Ms=1e6):
    """A uniform chain of N1 x 2 x 1 cubic cells along x (easy axis +z,
    alpha 1) holding a wall in the plane x = 0 at its middle: m = (0, sin,
    cos) of theta = 2 atan(exp(-(x - L/2) / sqrt(A / K)))."""
    n1 = int(round(length / hx))
    w = math.sqrt(A / K)
    x = np.arange(n1 + 1) * hx
    theta = 2.0 * np.arctan(np.exp(-(x - 0.5 * n1 * hx) / w))
    m = np.zeros((3, 2, 3, n1 + 1))
    m[1] = np.sin(theta)
    m[2] = np.cos(theta)
    p = make_problem((n1, 2, 1), (hx, hx, hx), Ms, A, 1.0, m0=(0.0, 0.0, 1.0), Ku=K, easy=(0.0, 0.0, 1.0))
    p["m0"] = _f32(m)
    return p
