"""Mesh, material and Q1 element matrices (oracle; test infrastructure only).

Follows Sec. 3.1 of the paper: cells c and nodes n = c + i with the local
vertex index i in {0,1}^3, trilinear nodal basis functions (Eq. nodal_basis)
and cell-wise constant material parameters (Eqs. ms_discrete, cell_basis).
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


class Mesh:
    """Regular cuboid grid of N1 x N2 x N3 cells of size h1 x h2 x h3 (Sec. 3.1)."""

    def __init__(self, n, h):
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        if min(self.n) < 1 or min(self.h) <= 0:
            raise ValueError("mesh needs n >= 1 and h > 0")
        self.V = self.h[0] * self.h[1] * self.h[2]

    @property
    def cell_shape(self):
        n1, n2, n3 = self.n
        return (n3, n2, n1)

    @property
    def node_shape(self):
        n1, n2, n3 = self.n
        return (n3 + 1, n2 + 1, n1 + 1)

    @property
    def n_cells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def n_nodes(self):
        return (self.n[0] + 1) * (self.n[1] + 1) * (self.n[2] + 1)

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
        """Exact element stiffness K^e and mass M^e of the Q1 basis, 8 x 8.

        K^e_ab = int_cell grad(phi_a) . grad(phi_b),  M^e_ab = int_cell phi_a phi_b,
        with phi the trilinear reference functions of Eq. (nodal_basis) scaled
        to the cell.  Both factor into 1D integrals per axis; 2-point Gauss
        quadrature per axis is exact for these integrands.
        """
        K = np.zeros((8, 8))
        M = np.zeros((8, 8))
        h = self.h
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
        for q in product(range(2), repeat=3):
            x = [g[q[0]], g[q[1]], g[q[2]]]
            wt = w[q[0]] * w[q[1]] * w[q[2]] * self.V
            for p, a in enumerate(CORNERS):
                for r, b in enumerate(CORNERS):
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

    def as_f64(self):
        def c(a):
            return None if a is None else np.asarray(a, dtype=np.float64)
        return Material(Ms=c(self.Ms), A=c(self.A), alpha=c(self.alpha),
                        gamma=float(self.gamma), Ku=c(self.Ku), easy=c(self.easy),
                        h_cell=c(self.h_cell), h_uniform=c(self.h_uniform),
                        drive_mask=c(self.drive_mask), drive_amp=c(self.drive_amp),
                        drive_freq=float(self.drive_freq),
                        drive_phase=float(self.drive_phase))
