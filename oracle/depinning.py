"""Domain-wall depinning at a planar phase boundary (oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.

The second validation case of the paper (Sec. "Validation", Tab. sp_dw)
pushes a domain wall from a soft phase into a hard phase and reports the
field at which it leaves the interface, for walls where A, K and Ms jump
across the boundary.  The system here is a chain of cells along x (m
uniform across it), soft phase then hard phase, uniaxial anisotropy along z in both, a uniform field
-H z, and exchange + anisotropy + Zeeman (no demag, as in the one-dimensional
model the closed form describes).  Two routes to the depinning field:

* `closed_form_field` -- the continuum limit.  With theta the angle of m from
  +z, the wall has theta -> pi in phase 1 (along the field) and theta -> 0 in
  phase 2.  Each phase has the first integral A theta'^2 = e(theta) with
    e1 = K1 sin^2 + mu0 Ms1 H (1 + cos),  e2 = K2 sin^2 - mu0 Ms2 H (1 - cos),
  and the weak form makes A theta' continuous at the interface, so the
  interface angle solves A1 e1 = A2 e2.  With u = 1 - cos(theta_0) that is
    -D u^2 + (2D - b (A2 Ms2 - A1 Ms1)) u - 2 b A1 Ms1 = 0,
  D = A2 K2 - A1 K1, b = mu0 H; the wall is pinned while a root u in (0, 2)
  exists.  The largest such b is where the discriminant vanishes,
    (2D - b (A2 Ms2 - A1 Ms1))^2 = 8 D A1 Ms1 b,
  whose smaller root is b = (2 K2 / Ms2) (1 - eK eA) / (1 + sqrt(eA eM))^2
  with eA = A1/A2, eK = K1/K2, eM = Ms1/Ms2 (the classical result for an
  abrupt interface).

* `discrete_depinning_field` -- the same threshold for the nodal
  discretisation: the largest field at which the discrete energy (the
  oracle's own, Sec. 3.1) still has a local minimum with the wall at the
  interface, found by bisection over H with quasi-static warm starts and
  float64 energy minimisation.  By the symmetry of the problem (no term
  prefers a rotation plane) the minimiser turns in one plane, so
  m = (0, sin theta, cos theta) with one angle per node column.
"""
import dataclasses

import numpy as np
from scipy.optimize import minimize

from .field import ANISOTROPY, EXCHANGE, ZEEMAN, energies, gradient
from .mesh import MU0

TERMS = EXCHANGE | ANISOTROPY | ZEEMAN


def closed_form_field(p1, p2):
    """mu0 H_p in T for an abrupt interface (continuum limit);
    p1 = (A1, K1, Ms1) of the soft phase, p2 of the hard phase."""
    (A1, K1, M1), (A2, K2, M2) = p1, p2
    eA, eK, eM = A1 / A2, K1 / K2, M1 / M2
    return 2.0 * K2 / M2 * (1.0 - eK * eA) / (1.0 + np.sqrt(eA * eM)) ** 2


def interface_angle(p1, p2, b):
    """theta_0 at the interface of the pinned wall at mu0 H = b < mu0 H_p:
    the smaller root u = 1 - cos(theta_0) of the interface condition (the
    stable wall; the larger root is the saddle it has to pass, and the two
    merge at the depinning field)."""
    (A1, K1, M1), (A2, K2, M2) = p1, p2
    D = A2 * K2 - A1 * K1
    B = 2 * D - b * (A2 * M2 - A1 * M1)
    disc = B * B - 8 * D * A1 * M1 * b
    if disc < 0:
        raise ValueError("no pinned wall at this field")
    u = (B - np.sqrt(disc)) / (2 * D)
    return float(np.arccos(1.0 - u))


def column_angles(m):
    """theta per node column of a chain magnetisation in the plane x = 0."""
    return np.arctan2(m[1, 0, 0], m[2, 0, 0])


def _m_of(mesh, theta):
    m = np.zeros((3,) + mesh.node_shape)
    m[1] = np.sin(theta)[None, None, :]
    m[2] = np.cos(theta)[None, None, :]
    return m


def _with_field(mat, b):
    """The material under mu0 H = b (T) along -z."""
    return dataclasses.replace(mat, h_uniform=np.array([0.0, 0.0, -b / MU0]))


def relax(mesh, mat, theta, b, gtol=1e-12):
    """Local minimum of the discrete energy reached from theta at mu0 H = b."""
    matb = _with_field(mat, b)
    scale = 1.0 / (float(np.max(mat.Ku)) * mesh.V * mesh.n_cells)

    def f(th):
        m = _m_of(mesh, th)
        e = energies(mesh, matb, m, TERMS)
        g = gradient(mesh, matb, m, TERMS)
        dth = np.sum(g[1] * np.cos(th)[None, None, :] - g[2] * np.sin(th)[None, None, :], axis=(0, 1))
        return (e["exchange"] + e["anisotropy"] + e["zeeman"]) * scale, dth * scale

    res = minimize(f, theta, jac=True, method="L-BFGS-B",
                   options={"gtol": gtol, "ftol": 0.0, "maxiter": 200000, "maxcor": 30})
    return res.x


def depinned(theta, n_soft):
    """The wall has left the interface: the hard phase is mostly reversed."""
    return float(np.mean(np.cos(theta[n_soft:]))) < 0.0


def discrete_depinning_field(mesh, mat, m0, n_soft, b_lo, b_hi, rel_tol=1e-3):
    """(b_lo, b_hi) in T bracketing the discrete depinning field of the chain
    (soft phase on its first n_soft cells): the wall, relaxed from m0, is
    still pinned at b_lo and has left at b_hi, b_hi - b_lo <= rel_tol b_hi."""
    theta = relax(mesh, mat, column_angles(np.asarray(m0, dtype=np.float64)), b_lo)
    if depinned(theta, n_soft):
        raise RuntimeError("wall not pinned at the lower end of the bracket")
    if not depinned(relax(mesh, mat, theta, b_hi), n_soft):
        raise RuntimeError("wall still pinned at the upper end of the bracket")
    lo, hi = b_lo, b_hi
    while hi - lo > rel_tol * hi:
        mid = 0.5 * (lo + hi)
        t = relax(mesh, mat, theta, mid)
        if depinned(t, n_soft):
            hi = mid
        else:
            lo, theta = mid, t
    return lo, hi
