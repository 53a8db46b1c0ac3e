"""Demagnetisation tensor of homogeneously magnetised cuboid cells (oracle).

Sec. 3.2 of the paper computes the demagnetisation field with the standard
finite-difference method: every cell is a homogeneously magnetised cuboid and
the cell-averaged field is H_c = -sum_c' N(c - c') M_c'.  The paper only cites
the tensor; it is computed here from its published closed form (Newell,
Williams and Dunlop, J. Geophys. Res. 98 (1993) 9551): N = D f / (4 pi V)
with D the 27-point second difference over the cell size and f, g the
Newell potentials.  That form cancels catastrophically at large distance
(about (r/h)^6 digits lost), so beyond a switch radius the oracle uses the
exact integral definition instead,

    N(X) = int_{[-h,h]^3} prod_k (1 - |u_k|/h_k) N_dip(X + u) du,
    N_dip(r) = (delta_ij r^2 - 3 r_i r_j) / (4 pi r^5),

(the cell-pair average of the point-dipole kernel, smooth once the cells are
apart) by tensor Gauss-Legendre quadrature on each half of every axis.

Component order everywhere: xx, yy, zz, xy, xz, yz.
"""
import numpy as np

# switch radius (in units of the largest cell edge) and Gauss-Legendre points
# per half axis by distance band; chosen so both routes agree to ~1e-11
# relative at every band edge
NEWELL_RADIUS = 4.0
GL_BANDS = ((8.0, 7), (20.0, 5), (60.0, 4), (np.inf, 3))


def _safe_div(num, den):
    return num / np.where(den != 0, den, 1.0)


def newell_f(x, y, z):
    """Newell potential f for the diagonal components (even in x, y and z)."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = (2.0 * x2 - y2 - z2) * R / 6.0
    rxz = np.sqrt(x2 + z2)
    out = out + np.where(rxz > 0, 0.5 * y * (z2 - x2) * np.arcsinh(_safe_div(y, rxz)), 0.0)
    rxy = np.sqrt(x2 + y2)
    out = out + np.where(rxy > 0, 0.5 * z * (y2 - x2) * np.arcsinh(_safe_div(z, rxy)), 0.0)
    out = out - np.where(x != 0, x * y * z * np.arctan(_safe_div(y * z, x * R)), 0.0)
    return out


def newell_g(x, y, z):
    """Newell potential g for the off-diagonal xy component (odd in x and y)."""
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    out = -x * y * R / 3.0
    rxy = np.sqrt(x2 + y2)
    out = out + np.where(rxy > 0, x * y * z * np.arcsinh(_safe_div(z, rxy)), 0.0)
    ryz = np.sqrt(y2 + z2)
    out = out + np.where(ryz > 0, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(_safe_div(x, ryz)), 0.0)
    rxz = np.sqrt(x2 + z2)
    out = out + np.where(rxz > 0, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(_safe_div(y, rxz)), 0.0)
    out = out - np.where(z != 0, z ** 3 / 6.0 * np.arctan(_safe_div(x * y, z * R)), 0.0)
    out = out - np.where(y != 0, z * y2 / 2.0 * np.arctan(_safe_div(x * z, y * R)), 0.0)
    out = out - np.where(x != 0, z * x2 / 2.0 * np.arctan(_safe_div(y * z, x * R)), 0.0)
    return out


def _second_difference(F, X, Y, Z, h):
    """sum over e in {-1,0,1}^3 of prod_k c(e_k) F(X + e h), c(0)=2, c(+-1)=-1."""
    c = {-1: -1.0, 0: 2.0, 1: -1.0}
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for e1 in (-1, 0, 1):
        for e2 in (-1, 0, 1):
            for e3 in (-1, 0, 1):
                w = c[e1] * c[e2] * c[e3]
                acc = acc + w * F(X + e1 * h[0], Y + e2 * h[1], Z + e3 * h[2])
    return acc


def newell_near(X, Y, Z, h):
    """All six components from the Newell closed form; X, Y, Z are offsets in
    length units (any scale: the result is scale invariant)."""
    V = h[0] * h[1] * h[2]
    s = 1.0 / (4.0 * np.pi * V)
    xx = _second_difference(newell_f, X, Y, Z, h)
    yy = _second_difference(lambda a, b, c: newell_f(b, a, c), X, Y, Z, h)
    zz = _second_difference(lambda a, b, c: newell_f(c, b, a), X, Y, Z, h)
    xy = _second_difference(newell_g, X, Y, Z, h)
    xz = _second_difference(lambda a, b, c: newell_g(a, c, b), X, Y, Z, h)
    yz = _second_difference(lambda a, b, c: newell_g(b, c, a), X, Y, Z, h)
    return s * np.stack([xx, yy, zz, xy, xz, yz])


def dipole_tensor(X, Y, Z):
    """Point-dipole kernel (delta r^2 - 3 r r^T) / (4 pi r^5) (six components)."""
    r2 = X * X + Y * Y + Z * Z
    k = 1.0 / (4.0 * np.pi * r2 ** 2.5)
    return k * np.stack([r2 - 3 * X * X, r2 - 3 * Y * Y, r2 - 3 * Z * Z,
                         -3 * X * Y, -3 * X * Z, -3 * Y * Z])


def _tent_rule(npts, hk):
    """Nodes/weights of int_{-hk}^{hk} (1 - |u|/hk) q(u) du, split at u = 0."""
    t, w = np.polynomial.legendre.leggauss(npts)
    u = 0.5 * (t + 1.0) * hk                  # nodes on [0, hk]
    wu = 0.5 * w * hk * (1.0 - u / hk)
    return np.concatenate([-u, u]), np.concatenate([wu, wu])


def newell_far(X, Y, Z, h, npts):
    """Tent-weighted Gauss-Legendre integral of the dipole kernel (see module doc)."""
    u1, w1 = _tent_rule(npts, h[0])
    u2, w2 = _tent_rule(npts, h[1])
    u3, w3 = _tent_rule(npts, h[2])
    out = np.zeros((6,) + np.broadcast(X, Y, Z).shape)
    X, Y, Z = np.broadcast_arrays(X, Y, Z)
    for a, wa in zip(u1, w1):
        for b, wb in zip(u2, w2):
            for c, wc in zip(u3, w3):
                out += (wa * wb * wc) * dipole_tensor(X + a, Y + b, Z + c)
    return out


def newell_offset(d, h):
    """N(d) for integer cell offsets d = (d1, d2, d3) arrays (any sign)."""
    d1, d2, d3 = (np.asarray(v, dtype=np.float64) for v in d)
    hs = max(h)
    hh = tuple(v / hs for v in h)            # scale-free units
    X, Y, Z = np.broadcast_arrays(d1 * hh[0], d2 * hh[1], d3 * hh[2])
    rho = np.sqrt(X * X + Y * Y + Z * Z)     # distance in largest-edge units
    out = np.zeros((6,) + X.shape)
    near = rho < NEWELL_RADIUS
    if near.any():
        out[:, near] = newell_near(X[near], Y[near], Z[near], hh)
    lo = NEWELL_RADIUS
    for hi, npts in GL_BANDS:
        sel = (rho >= lo) & (rho < hi)
        if sel.any():
            out[:, sel] = newell_far(X[sel], Y[sel], Z[sel], hh, npts)
        lo = hi
    return out


def newell_octant(n, h):
    """N(d) on the non-negative octant 0 <= d_k < N_k; shape (6, N3, N2, N1).

    Negative offsets follow from the parities: the diagonal components are
    even in every axis, xy is odd in x and y, xz odd in x and z, yz odd in y
    and z (each even in the remaining axis).
    """
    n1, n2, n3 = n
    d3, d2, d1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    out = np.empty((6, n3, n2, n1))
    flat = [d1.ravel(), d2.ravel(), d3.ravel()]
    chunk = 20000
    for s in range(0, flat[0].size, chunk):
        blk = newell_offset([f[s:s + chunk] for f in flat], h)
        out.reshape(6, -1)[:, s:s + chunk] = blk
    return out
