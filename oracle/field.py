"""Effective field and energies of the nodal discretisation (oracle).

Everything here follows Sec. 3 of the paper step by step, in float64:

* gradient g_n = dE/dm_n is assembled cell by cell with the shifted slices of
  Eqs. (weak_form_impl_f) and (weak_form_impl): for every local vertex pair
  (a, b) of the 8 x 8 element matrix, the cell contribution is added to the
  node c + a;
* the field follows from mass lumping, Eq. (mass_lumping):
  H_n = -g_n / M_n with M_n = int mu0 Ms^h phi_n = mu0 sum_{c containing n} Ms_c V/8
  (V/4 under the thin-film basis, whose cells have 4 local vertices);
* demagnetisation (Sec. 3.2): nodal m is averaged to cells, convolved with
  the cuboid tensor by FFT (zero padded), and the cell field is brought back
  to the nodes through the same lumped weak form.

Energies (J):
  exchange   E_ex = sum_c A_c sum_j m_j^T K^e m_j            (Eq. exchange_energy)
  anisotropy E_an = -sum_c Ku_c sum_ab M^e_ab (m_a.e_c)(m_b.e_c)
  Zeeman     E_z  = -mu0 sum_c Ms_c V/8 H_ext,c . sum_a m_{c+a}
  demag      E_d  = -(mu0/2) sum_c V Ms_c mbar_c . H_c
  DMI        interfacial (the interface normal along z):
             E_dmi = sum_c D_c int_c [m_z div m - (m . grad) m_z];
             bulk: E_dmi = sum_c D_c int_c m . (curl m);
             both antisymmetric exchange (Sec. 2), integrated exactly with
             the element matrices G_k[a, b] = int phi_a d_k phi_b
  cubic      E_c = sum_c Kc_c int_c (a1^2 a2^2 + a2^2 a3^2 + a3^2 a1^2),
             a_i = m^h . c_i with the cell's cubic axes c1, c2, c3 = c1 x c2;
             quartic in m, integrated by the 2-point Gauss rule per axis (the
             form compiler's quadrature of the integrand, Sec. 5.1; the rule
             that is exact for every quadratic term of the Q1 functions)
"""
import numpy as np

from .mesh import MU0
from .newell import newell_octant

EXCHANGE, DEMAG, ANISOTROPY, ZEEMAN, DMI, CUBIC = 1, 2, 4, 8, 16, 32
ALL_TERMS = 63


# ---------------------------------------------------------------------------
# mass, nodal coefficients, external field
# ---------------------------------------------------------------------------
def lumped_mass(mesh, mat):
    """M_n = mu0 sum_{c containing n} Ms_c V / 8  (Eq. mass_lumping; V / 4 for
    the 4 vertices of a film-basis cell)."""
    M = np.zeros(mesh.node_shape)
    for a in mesh.corners:
        mesh.corner(M, a)[...] += MU0 * mat.Ms * mesh.V / len(mesh.corners)
    return M


def nodal_alpha(mesh, mat):
    """Ms-weighted mean of the cell damping over the cells sharing a node."""
    num = np.zeros(mesh.node_shape)
    den = np.zeros(mesh.node_shape)
    for a in mesh.corners:
        mesh.corner(num, a)[...] += mat.Ms * mat.alpha
        mesh.corner(den, a)[...] += mat.Ms
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def external_cell_field(mesh, mat, t):
    """Applied field per cell at time t (A/m), shape (3, N3, N2, N1)."""
    H = np.zeros((3,) + mesh.cell_shape)
    H += np.asarray(mat.h_uniform, dtype=np.float64).reshape(3, 1, 1, 1)
    if mat.h_cell is not None:
        H += mat.h_cell
    if mat.drive_mask is not None:
        s = np.sin(2.0 * np.pi * mat.drive_freq * t + mat.drive_phase)
        H += (np.asarray(mat.drive_amp, dtype=np.float64).reshape(3, 1, 1, 1)
              * mat.drive_mask[None] * s)
    return H


# ---------------------------------------------------------------------------
# local terms
# ---------------------------------------------------------------------------
def _exchange_gradient(mesh, mat, m, g):
    K, _ = mesh.element_matrices()
    for p, a in enumerate(mesh.corners):
        acc = np.zeros((3,) + mesh.cell_shape)
        for q, b in enumerate(mesh.corners):
            acc += K[p, q] * mesh.corner(m, b)
        mesh.corner(g, a)[...] += 2.0 * mat.A * acc


def _anisotropy_gradient(mesh, mat, m, g):
    _, Me = mesh.element_matrices()
    e = mat.easy
    proj = [np.einsum("jzyx,jzyx->zyx", mesh.corner(m, b), e) for b in mesh.corners]
    for p, a in enumerate(mesh.corners):
        acc = np.zeros(mesh.cell_shape)
        for q in range(len(mesh.corners)):
            acc += Me[p, q] * proj[q]
        mesh.corner(g, a)[...] += -2.0 * mat.Ku * acc * e


def _dmi_gradient(mesh, mat, m, g):
    """dE/dm of the DMI energy, with A_k = G_k - G_k^T.

    Interfacial: E = sum_c D_c sum_ab [m_az G_x m_bx - m_ax G_x m_bz
    + m_az G_y m_by - m_ay G_y m_bz] (G = G_k[a, b]):
        dE/dm_a,x = -sum_b A_x[a, b] m_b,z,  dE/dm_a,y = -sum_b A_y[a, b] m_b,z,
        dE/dm_a,z = sum_b (A_x[a, b] m_b,x + A_y[a, b] m_b,y).
    Bulk: E = sum_c D_c sum_ab eps_jkl m_aj G_k[a, b] m_bl:
        dE/dm_a,j = sum_b eps_jkl A_k[a, b] m_b,l."""
    G = mesh.element_first_derivative()
    A = [G[k] - G[k].T for k in range(3)]
    for p, a in enumerate(mesh.corners):
        acc = np.zeros((3,) + mesh.cell_shape)
        for q, b in enumerate(mesh.corners):
            mb = mesh.corner(m, b)
            if mat.dmi_type == "bulk":
                for j in range(3):
                    k, l = (j + 1) % 3, (j + 2) % 3
                    acc[j] += A[k][p, q] * mb[l] - A[l][p, q] * mb[k]
            else:
                acc[0] -= A[0][p, q] * mb[2]
                acc[1] -= A[1][p, q] * mb[2]
                acc[2] += A[0][p, q] * mb[0] + A[1][p, q] * mb[1]
        mesh.corner(g, a)[...] += mat.D * acc


def _cubic_axes(mat):
    c1, c2 = mat.cubic[0], mat.cubic[1]
    return c1, c2, np.cross(c1, c2, axis=0)


def cubic_density_gradient(mc, axes):
    """f = a1^2 a2^2 + a2^2 a3^2 + a3^2 a1^2 (a_i = m . c_i) and df/dm
    = sum_i 2 a_i (a_j^2 + a_k^2) c_i, for (3, ...) arrays."""
    a = [np.sum(mc * c, axis=0) for c in axes]
    f = a[0] ** 2 * a[1] ** 2 + a[1] ** 2 * a[2] ** 2 + a[2] ** 2 * a[0] ** 2
    df = sum(2.0 * a[i] * (a[(i + 1) % 3] ** 2 + a[(i + 2) % 3] ** 2) * axes[i] for i in range(3))
    return f, df


def _cubic_gradient(mesh, mat, m, g):
    """dE/dm_a = sum_g w_g phi_a(x_g) Kc df/dm(m^h(x_g)) over the 2-point
    Gauss points of each cell, m^h(x_g) = sum_b phi_b(x_g) m_b."""
    axes = _cubic_axes(mat)
    corners = [mesh.corner(m, b) for b in mesh.corners]
    for w, phi in mesh.gauss_points():
        mg = sum(phi[q] * corners[q] for q in range(len(corners)))
        _, df = cubic_density_gradient(mg, axes)
        for p, a in enumerate(mesh.corners):
            mesh.corner(g, a)[...] += w * phi[p] * mat.Kc * df


def _cell_source_gradient(mesh, mat, Hc, g):
    """Gradient of -mu0 int Ms m^h . H for a cell-wise constant field H."""
    w = -MU0 * mat.Ms * mesh.V / len(mesh.corners)
    for a in mesh.corners:
        mesh.corner(g, a)[...] += w * Hc


# ---------------------------------------------------------------------------
# demagnetisation
# ---------------------------------------------------------------------------
def cell_average(mesh, m):
    """mbar_c = (1/8) sum_i m_{c+i} (1/4 under the film basis): the exact cell
    mean of the nodal m^h."""
    acc = np.zeros(m.shape[:-3] + mesh.cell_shape)
    for a in mesh.corners:
        acc += mesh.corner(m, a)
    return acc / len(mesh.corners)


_SIGNS = {  # parity of each component under d_k -> -d_k, axes (x, y, z)
    0: (1, 1, 1), 1: (1, 1, 1), 2: (1, 1, 1),
    3: (-1, -1, 1), 4: (-1, 1, -1), 5: (1, -1, -1),
}


def _offset_tensor(octant, n):
    """N(d) on all offsets -(N_k-1) <= d_k <= N_k-1, shape (6, 2N3-1, 2N2-1, 2N1-1)."""
    n1, n2, n3 = n
    out = np.empty((6, 2 * n3 - 1, 2 * n2 - 1, 2 * n1 - 1))
    d1 = np.arange(-(n1 - 1), n1)
    d2 = np.arange(-(n2 - 1), n2)
    d3 = np.arange(-(n3 - 1), n3)
    for comp in range(6):
        sx, sy, sz = _SIGNS[comp]
        base = octant[comp][np.ix_(np.abs(d3), np.abs(d2), np.abs(d1))]
        fx = np.where(d1 < 0, sx, 1)[None, None, :]
        fy = np.where(d2 < 0, sy, 1)[None, :, None]
        fz = np.where(d3 < 0, sz, 1)[:, None, None]
        out[comp] = base * fx * fy * fz
    return out


def padded_tensor(octant, n, pad):
    """Real-space tensor on the periodic padded grid P (pad), shape (6, P3, P2, P1).

    Offset d lands at index d mod P_k; offsets that do not occur (|d_k| >= N_k)
    are zero, which turns the cyclic convolution into the linear one whenever
    P_k >= 2 N_k - 1."""
    n1, n2, n3 = n
    p1, p2, p3 = pad
    full = _offset_tensor(octant, n)
    out = np.zeros((6, p3, p2, p1))
    i1 = np.arange(-(n1 - 1), n1) % p1
    i2 = np.arange(-(n2 - 1), n2) % p2
    i3 = np.arange(-(n3 - 1), n3) % p3
    out[np.ix_(range(6), i3, i2, i1)] = full
    return out


def default_padding(n):
    return tuple(2 * v if v > 1 else 1 for v in n)


_TENSOR_CACHE = {}
_SPECTRUM_CACHE = {}


def demag_octant(mesh):
    key = (mesh.n, mesh.h)
    if key not in _TENSOR_CACHE:
        _TENSOR_CACHE[key] = newell_octant(mesh.n, mesh.h)
    return _TENSOR_CACHE[key]


def demag_cell_field(mesh, mat, m, pad=None, octant=None):
    """H_c = -sum_c' N(c - c') Ms_c' mbar_c' by zero-padded FFT convolution."""
    n1, n2, n3 = mesh.n
    pad = default_padding(mesh.n) if pad is None else tuple(pad)
    if any(p < 2 * v - 1 for p, v in zip(pad, mesh.n)):
        raise ValueError("padding must satisfy P_k >= 2 N_k - 1")
    if octant is None:
        key = (mesh.n, mesh.h, pad)
        if key not in _SPECTRUM_CACHE:
            _SPECTRUM_CACHE[key] = np.fft.fftn(
                padded_tensor(demag_octant(mesh), mesh.n, pad), axes=(1, 2, 3))
        Nk = _SPECTRUM_CACHE[key]
    else:
        Nk = np.fft.fftn(padded_tensor(octant, mesh.n, pad), axes=(1, 2, 3))
    Mc = mat.Ms * cell_average(mesh, m)
    Mp = np.zeros((3, pad[2], pad[1], pad[0]))
    Mp[:, :n3, :n2, :n1] = Mc
    Mk = np.fft.fftn(Mp, axes=(1, 2, 3))
    xx, yy, zz, xy, xz, yz = Nk
    Hk = -np.stack([xx * Mk[0] + xy * Mk[1] + xz * Mk[2],
                    xy * Mk[0] + yy * Mk[1] + yz * Mk[2],
                    xz * Mk[0] + yz * Mk[1] + zz * Mk[2]])
    H = np.fft.ifftn(Hk, axes=(1, 2, 3)).real
    return H[:, :n3, :n2, :n1]


def demag_cell_field_direct(mesh, mat, m, octant=None):
    """The same cell field by the brute-force double sum over cell pairs."""
    n1, n2, n3 = mesh.n
    octant = demag_octant(mesh) if octant is None else octant
    T = _offset_tensor(octant, mesh.n)
    Mc = mat.Ms * cell_average(mesh, m)
    H = np.zeros((3,) + mesh.cell_shape)
    for c3 in range(n3):
        for c2 in range(n2):
            for c1 in range(n1):
                # offsets c - c' for all target cells c
                blk = T[:, n3 - 1 - c3:2 * n3 - 1 - c3, n2 - 1 - c2:2 * n2 - 1 - c2,
                        n1 - 1 - c1:2 * n1 - 1 - c1]
                mx, my, mz = Mc[:, c3, c2, c1]
                xx, yy, zz, xy, xz, yz = blk
                H[0] -= xx * mx + xy * my + xz * mz
                H[1] -= xy * mx + yy * my + yz * mz
                H[2] -= xz * mx + yz * my + zz * mz
    return H


# ---------------------------------------------------------------------------
# field and energy
# ---------------------------------------------------------------------------
def gradient(mesh, mat, m, terms=ALL_TERMS, t=0.0, pad=None):
    """g_n,j = dE/dm_n,j summed over the selected terms."""
    m = np.asarray(m, dtype=np.float64)
    g = np.zeros((3,) + mesh.node_shape)
    if terms & EXCHANGE:
        _exchange_gradient(mesh, mat, m, g)
    if terms & ANISOTROPY and mat.Ku is not None:
        _anisotropy_gradient(mesh, mat, m, g)
    if terms & DMI and mat.D is not None:
        _dmi_gradient(mesh, mat, m, g)
    if terms & CUBIC and mat.Kc is not None:
        _cubic_gradient(mesh, mat, m, g)
    if terms & ZEEMAN:
        _cell_source_gradient(mesh, mat, external_cell_field(mesh, mat, t), g)
    if terms & DEMAG:
        _cell_source_gradient(mesh, mat, demag_cell_field(mesh, mat, m, pad=pad), g)
    return g


def heff(mesh, mat, m, terms=ALL_TERMS, t=0.0, pad=None):
    """Nodal effective field H_n = -g_n / M_n (Eq. mass_lumping); zero where M_n = 0."""
    g = gradient(mesh, mat, m, terms, t, pad)
    M = lumped_mass(mesh, mat)
    return np.where(M > 0, -g / np.where(M > 0, M, 1.0), 0.0)


def energies(mesh, mat, m, terms=ALL_TERMS, t=0.0):
    """Energies in J as a dict: exchange, demag, anisotropy, zeeman, total."""
    m = np.asarray(m, dtype=np.float64)
    K, Me = mesh.element_matrices()
    out = {"exchange": 0.0, "demag": 0.0, "anisotropy": 0.0, "zeeman": 0.0, "dmi": 0.0, "cubic": 0.0}
    if terms & EXCHANGE:
        e = 0.0
        for p, a in enumerate(mesh.corners):
            ma = mesh.corner(m, a)
            for q, b in enumerate(mesh.corners):
                e += K[p, q] * np.sum(mat.A * np.sum(ma * mesh.corner(m, b), axis=0))
        out["exchange"] = e
    if terms & ANISOTROPY and mat.Ku is not None:
        proj = [np.sum(mesh.corner(m, a) * mat.easy, axis=0) for a in mesh.corners]
        e = 0.0
        for p in range(len(mesh.corners)):
            for q in range(len(mesh.corners)):
                e -= Me[p, q] * np.sum(mat.Ku * proj[p] * proj[q])
        out["anisotropy"] = e
    if terms & ZEEMAN:
        H = external_cell_field(mesh, mat, t)
        msum = len(mesh.corners) * cell_average(mesh, m)
        out["zeeman"] = -MU0 * np.sum(mat.Ms * mesh.V / len(mesh.corners) * np.sum(H * msum, axis=0))
    if terms & DEMAG:
        Hc = demag_cell_field(mesh, mat, m)
        mbar = cell_average(mesh, m)
        out["demag"] = -0.5 * MU0 * mesh.V * np.sum(mat.Ms * np.sum(mbar * Hc, axis=0))
    if terms & DMI and mat.D is not None:
        G = mesh.element_first_derivative()
        e = 0.0
        for p, a in enumerate(mesh.corners):
            ma = mesh.corner(m, a)
            for q, b in enumerate(mesh.corners):
                mb = mesh.corner(m, b)
                if mat.dmi_type == "bulk":
                    # eps_jkl m_aj G_k m_bl
                    e += np.sum(mat.D * sum(G[(j + 1) % 3, p, q] * ma[j] * mb[(j + 2) % 3]
                                            - G[(j + 2) % 3, p, q] * ma[j] * mb[(j + 1) % 3]
                                            for j in range(3)))
                else:
                    e += np.sum(mat.D * (G[0, p, q] * (ma[2] * mb[0] - ma[0] * mb[2])
                                         + G[1, p, q] * (ma[2] * mb[1] - ma[1] * mb[2])))
        out["dmi"] = e
    if terms & CUBIC and mat.Kc is not None:
        axes = _cubic_axes(mat)
        corners = [mesh.corner(m, b) for b in mesh.corners]
        e = 0.0
        for w, phi in mesh.gauss_points():
            f, _ = cubic_density_gradient(sum(phi[q] * corners[q] for q in range(len(corners))), axes)
            e += w * np.sum(mat.Kc * f)
        out["cubic"] = e
    out["total"] = (out["exchange"] + out["demag"] + out["anisotropy"] + out["zeeman"] + out["dmi"]
                    + out["cubic"])
    return out
