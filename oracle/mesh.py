"""Mesh, material and Q1 element matrices (oracle; test infrastructure only).

Follows Sec. 3.1 of the paper: cells c and nodes n = c + i with the local
vertex index i in {0,1}^3, trilinear nodal basis functions (Eq. nodal_basis)
and cell-wise constant material parameters (Eqs. ms_discrete, cell_basis).

The thin-film basis of Sec. 3.3 (low-dimensional geometries) keeps the
in-plane bilinear functions and makes them constant along z, with the weak
form still integrated over the full cell: a single layer of cells then
carries one layer of (N1 + 1) x (N2 + 1) nodes, and a cell has the 4 local
vertices (i1, i2, 0).
"""
from dataclasses import dataclass, field
from itertools import product
from typing import Optional

import numpy as np

# mu0 fixed to 4*pi*1e-7 exactly (the pre-2019 SI value); the same value is
# used by the GPU library so that both start from identical constants.
MU0 = 4.0e-7 * np.pi

# the 8 local vertices i = (i1, i2, i3) of a cell, i1 varies fastest
CORNERS = [(i1, i2, i3) for i3 in (0, 1) for i2 in (0, 1) for i1 in (0, 1)]


# the 4 local vertices of a cell under the thin-film basis (constant along z)
FILM_CORNERS = [(i1, i2, 0) for i2 in (0, 1) for i1 in (0, 1)]


class Mesh:
    """Regular cuboid grid of N1 x N2 x N3 cells of size h1 x h2 x h3 (Sec. 3.1).

    basis "3d": trilinear nodal functions, (N1+1)(N2+1)(N3+1) nodes;
    basis "film": bilinear in-plane functions constant along z (Sec. 3.3),
    one cell layer (N3 = 1) and (N1+1)(N2+1) nodes.
    """

    def __init__(self, n, h, basis="3d"):
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        if min(self.n) < 1 or min(self.h) <= 0:
            raise ValueError("mesh needs n >= 1 and h > 0")
        if basis not in ("3d", "film"):
            raise ValueError("basis is '3d' or 'film'")
        if basis == "film" and self.n[2] != 1:
            raise ValueError("the film basis takes one layer of cells")
        self.basis = basis
        self.corners = CORNERS if basis == "3d" else FILM_CORNERS
        self.V = self.h[0] * self.h[1] * self.h[2]

    @property
    def cell_shape(self):
        n1, n2, n3 = self.n
        return (n3, n2, n1)

    @property
    def node_shape(self):
        n1, n2, n3 = self.n
        return (n3 + 1 if self.basis == "3d" else 1, n2 + 1, n1 + 1)

    @property
    def n_cells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def n_nodes(self):
        return int(np.prod(self.node_shape))

    def corner(self, f, i):
        """View of a nodal array at the nodes c + i of every cell c.

        Realises the shifted slicing of Eq. (weak_form_impl_f): for local
        vertex i the node of cell c is n = c + i.
        """
        n1, n2, n3 = self.n
        i1, i2, i3 = i
        return f[..., i3:i3 + n3, i2:i2 + n2, i1:i1 + n1]

    # --- element matrices -------------------------------------------------
    def element_matrices(self):
        """Exact element stiffness K^e and mass M^e, one row per local vertex.

        K^e_ab = int_cell grad(phi_a) . grad(phi_b),  M^e_ab = int_cell phi_a phi_b,
        with phi the trilinear reference functions of Eq. (nodal_basis) scaled
        to the cell.  Both factor into 1D integrals per axis; 2-point Gauss
        quadrature per axis is exact for these integrands.  Under the film
        basis the z factor is constant: its integral is h3 and its derivative
        vanishes.
        """
        nc = len(self.corners)
        K = np.zeros((nc, nc))
        M = np.zeros((nc, nc))
        h = self.h
        if self.basis == "film":
            for p, a in enumerate(self.corners):
                for q, b in enumerate(self.corners):
                    mx, my = (h[k] * (2.0 if a[k] == b[k] else 1.0) / 6.0 for k in range(2))
                    sx, sy = ((1.0 if a[k] == b[k] else -1.0) / h[k] for k in range(2))
                    K[p, q] = (sx * my + mx * sy) * h[2]
                    M[p, q] = mx * my * h[2]
            return K, M
        # 1D integrals on [0, hk] of the two linear hat pieces
        def s1(a, b, hk):  # int phi_a' phi_b'
            return (1.0 if a == b else -1.0) / hk

        def m1(a, b, hk):  # int phi_a phi_b
            return hk * (2.0 if a == b else 1.0) / 6.0

        for p, a in enumerate(CORNERS):
            for q, b in enumerate(CORNERS):
                mm = [m1(a[k], b[k], h[k]) for k in range(3)]
                ss = [s1(a[k], b[k], h[k]) for k in range(3)]
                K[p, q] = (ss[0] * mm[1] * mm[2] + mm[0] * ss[1] * mm[2]
                           + mm[0] * mm[1] * ss[2])
                M[p, q] = mm[0] * mm[1] * mm[2]
        return K, M

    def element_dmi(self):
        """G_k[a, b] = int_cell phi_a d(phi_b)/dx_k for k = x, y (the
        interfacial antisymmetric-exchange element matrices)."""
        return self.element_first_derivative()[:2]

    def element_first_derivative(self):
        """G_k[a, b] = int_cell phi_a d(phi_b)/dx_k for k = x, y, z.  Along k
        the 1D integral of psi_a psi_b' is +-1/2 (the sign of psi_b'), the
        other axes give the 1D mass factors; under the film basis the z factor
        is h3 and the z derivative vanishes."""
        h = self.h
        nc = len(self.corners)
        G = np.zeros((3, nc, nc))
        for p, a in enumerate(self.corners):
            for q, b in enumerate(self.corners):
                for k in range(3 if self.basis == "3d" else 2):
                    v = 0.5 if b[k] == 1 else -0.5
                    for l in range(3):
                        if l == k:
                            continue
                        if l == 2 and self.basis == "film":
                            v *= h[2]
                        else:
                            v *= h[l] * (2.0 if a[l] == b[l] else 1.0) / 6.0
                    G[k, p, q] = v
        return G

    def element_dmi_quadrature(self):
        """The same G_k (k = x, y) by 2-point Gauss quadrature of the reference functions."""
        return self.element_first_derivative_quadrature()[:2]

    def element_first_derivative_quadrature(self):
        """G_k (k = x, y, z) by 2-point Gauss quadrature of the reference functions."""
        g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
        w = np.array([0.5, 0.5])
        dims = 3 if self.basis == "3d" else 2

        def psi(i, x):
            return 1 - i + (2 * i * x - x)

        def phi(i, x):
            return np.prod([psi(i[k], x[k]) for k in range(dims)])

        def dphi(i, x, k):
            out = (2 * i[k] - 1) / self.h[k]
            for l in range(dims):
                if l != k:
                    out *= psi(i[l], x[l])
            return out
        nc = len(self.corners)
        G = np.zeros((3, nc, nc))
        for q in product(range(2), repeat=3):
            x = [g[q[0]], g[q[1]], g[q[2]]]
            wt = w[q[0]] * w[q[1]] * w[q[2]] * self.V
            for p, a in enumerate(self.corners):
                for r, b in enumerate(self.corners):
                    for k in range(dims):
                        G[k, p, r] += wt * phi(a, x) * dphi(b, x, k)
        return G

    def gauss_points(self):
        """2-point Gauss rule per axis on a cell (Sec. 5.1: the form compiler
        integrates over the elements by Gauss quadrature): a list of
        (weight, [phi_a(x_g) for each local vertex a]); the weights sum to V.
        Under the film basis the functions are constant along z, whose points
        then coincide in pairs."""
        g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
        dims = 3 if self.basis == "3d" else 2
        out = []
        for q in product(range(2), repeat=3):
            x = [g[q[0]], g[q[1]], g[q[2]]]
            vals = [np.prod([(x[k] if a[k] else 1.0 - x[k]) for k in range(dims)]) for a in self.corners]
            out.append((self.V / 8.0, vals))
        return out

    def element_matrices_quadrature(self):
        """Same matrices by explicit 2-point Gauss quadrature (as the paper's form
        compiler does, Sec. 5.1); used by the tests as an independent route."""
        g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
        w = np.array([0.5, 0.5])
        K = np.zeros((8, 8))
        M = np.zeros((8, 8))

        def phi(i, x):  # reference basis of Eq. (nodal_basis) on [0,1]^3
            return np.prod([1 - i[k] + (2 * i[k] * x[k] - x[k]) for k in range(3)])

        def dphi(i, x, k):
            out = 1.0
            for l in range(3):
                if l == k:
                    out *= (2 * i[l] - 1)
                else:
                    out *= 1 - i[l] + (2 * i[l] * x[l] - x[l])
            return out

        h = self.h
        if self.basis == "film":
            # the 2D reference functions of Sec. 3.3, constant along x3
            def phi(i, x):
                return np.prod([1 - i[k] + (2 * i[k] * x[k] - x[k]) for k in range(2)])

            def dphi(i, x, k):
                if k == 2:
                    return 0.0
                out = 1.0
                for l in range(2):
                    out *= (2 * i[l] - 1) if l == k else 1 - i[l] + (2 * i[l] * x[l] - x[l])
                return out
            K = np.zeros((4, 4))
            M = np.zeros((4, 4))
        for q in product(range(2), repeat=3):
            x = [g[q[0]], g[q[1]], g[q[2]]]
            wt = w[q[0]] * w[q[1]] * w[q[2]] * self.V
            for p, a in enumerate(self.corners):
                for r, b in enumerate(self.corners):
                    M[p, r] += wt * phi(a, x) * phi(b, x)
                    K[p, r] += wt * sum(dphi(a, x, k) * dphi(b, x, k) / h[k] ** 2
                                        for k in range(3))
        return K, M


@dataclass
class Material:
    """Cell-wise material parameters (Eq. ms_discrete) and applied fields.

    All arrays are cell-shaped (N3, N2, N1) or (3, N3, N2, N1).  Units are SI:
    Ms and fields in A/m, A in J/m, Ku in J/m^3, gamma in m/(A s).
    External field on cell c at time t:
        h_uniform + h_cell[:, c] + drive_mask[c] * drive_amp * sin(2 pi f t + phase)
    """
    Ms: np.ndarray
    A: np.ndarray
    alpha: np.ndarray
    gamma: float = 2.211e5
    Ku: Optional[np.ndarray] = None
    easy: Optional[np.ndarray] = None
    h_cell: Optional[np.ndarray] = None
    h_uniform: np.ndarray = field(default_factory=lambda: np.zeros(3))
    drive_mask: Optional[np.ndarray] = None
    drive_amp: np.ndarray = field(default_factory=lambda: np.zeros(3))
    drive_freq: float = 0.0
    drive_phase: float = 0.0
    D: Optional[np.ndarray] = None      # DMI constant per cell, J/m^2
    dmi_type: str = "interfacial"       # or "bulk"
    Kc: Optional[np.ndarray] = None     # cubic anisotropy constant K1 per cell, J/m^3
    cubic: Optional[np.ndarray] = None  # cubic axes c1, c2 per cell, (2, 3, N3, N2, N1); c3 = c1 x c2

    def as_f64(self):
        def c(a):
            return None if a is None else np.asarray(a, dtype=np.float64)
        return Material(Ms=c(self.Ms), A=c(self.A), alpha=c(self.alpha),
                        gamma=float(self.gamma), Ku=c(self.Ku), easy=c(self.easy),
                        h_cell=c(self.h_cell), h_uniform=c(self.h_uniform),
                        drive_mask=c(self.drive_mask), drive_amp=c(self.drive_amp),
                        drive_freq=float(self.drive_freq),
                        drive_phase=float(self.drive_phase), D=c(self.D), dmi_type=self.dmi_type,
                        Kc=c(self.Kc), cubic=c(self.cubic))
