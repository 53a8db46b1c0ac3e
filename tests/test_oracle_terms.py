"""Pins of the oracle's further energy terms (Sec. 2 names antisymmetric
exchange and crystalline anisotropies as terms the method handles):

* bulk DMI, E = sum_c D_c int_c m . (curl m), through the first-derivative
  element matrices G_k[a, b] = int phi_a d_k phi_b (k = x, y, z);
* cubic anisotropy, E = sum_c Kc_c int_c (a1^2 a2^2 + a2^2 a3^2 + a3^2 a1^2)
  with a_i = m . c_i, integrated by the 2-point Gauss rule per axis.

Pins: element matrices against Gauss quadrature and their column sums, the
Gauss rule against the exact mass matrix, fields against finite differences
of the energies, an interior helix against the centred difference of the
continuum bulk-DMI field, the uniform-state closed form of the cubic field
and energy, its zero torque along the cubic axes and its symmetries.
"""
import numpy as np
import pytest

import oracle
from oracle.field import CUBIC, DMI, cubic_density_gradient

from helpers import rel_l2, to_oracle
from paper_2411_11725_amd import synth

MU0 = 4e-7 * np.pi


@pytest.mark.parametrize("basis", ["3d", "film"])
def test_first_derivative_element_matrices(basis):
    mesh = oracle.Mesh((1, 1, 1), (1.3e-9, 0.7e-9, 2.1e-9), basis=basis)
    G = mesh.element_first_derivative()
    Gq = mesh.element_first_derivative_quadrature()
    assert G.shape[0] == 3
    assert np.allclose(G, Gq, rtol=0, atol=1e-12 * np.abs(G).max())
    # sum over a of G_k[a, b] = int d_k phi_b = +-(face area)/4 along k (3D)
    for k in range(3 if basis == "3d" else 2):
        col = G[k].sum(axis=0)
        want = np.array([(1.0 if b[k] == 1 else -1.0) * mesh.V / mesh.h[k] for b in mesh.corners])
        want /= 4.0 if basis == "3d" else 2.0
        assert np.allclose(col, want, rtol=1e-12, atol=0)
    if basis == "film":
        assert not np.any(G[2])


@pytest.mark.parametrize("basis", ["3d", "film"])
def test_gauss_rule_integrates_basis_products_exactly(basis):
    """sum_g w_g phi_a(x_g) phi_b(x_g) = the exact mass matrix M^e; the
    weights sum to the cell volume."""
    mesh = oracle.Mesh((1, 1, 1), (1.3e-9, 0.7e-9, 2.1e-9), basis=basis)
    _, Me = mesh.element_matrices()
    pts = mesh.gauss_points()
    Mq = sum(w * np.outer(phi, phi) for w, phi in pts)
    assert abs(sum(w for w, _ in pts) - mesh.V) <= 1e-12 * mesh.V
    assert np.allclose(Mq, Me, rtol=1e-12, atol=0)


def _problem(seed, n=(5, 4, 3), basis="3d"):
    p = synth.small_random(n, (2e-9, 2.5e-9, 3e-9), seed=seed)
    if basis == "film":
        p = synth.as_film(synth.small_random((n[0], n[1], 1), (2e-9, 2.5e-9, 3e-9), seed=seed))
    mesh, mat, m0 = to_oracle(p)
    rng = np.random.default_rng(seed)
    mat.D = rng.uniform(-3e-3, 3e-3, size=mesh.cell_shape)
    mat.dmi_type = "bulk"
    mat.Kc = rng.uniform(-4e5, 4e5, size=mesh.cell_shape)
    c1 = synth.random_unit_vectors(mesh.n_cells, rng).reshape((3,) + mesh.cell_shape)
    r = synth.random_unit_vectors(mesh.n_cells, rng).reshape((3,) + mesh.cell_shape)
    c2 = np.cross(c1, r, axis=0)
    c2 /= np.linalg.norm(c2, axis=0, keepdims=True)
    mat.cubic = np.stack([c1, c2])
    return mesh, mat, m0


@pytest.mark.parametrize("term,key", [(DMI, "dmi"), (CUBIC, "cubic")])
@pytest.mark.parametrize("basis", ["3d", "film"])
def test_field_is_minus_energy_gradient_over_mass(term, key, basis):
    mesh, mat, m0 = _problem(93, basis=basis)
    H = oracle.heff(mesh, mat, m0, term)
    M = oracle.lumped_mass(mesh, mat)
    rng = np.random.default_rng(5)
    eps = 1e-6
    assert np.abs(H).max() > 0
    for _ in range(8):
        idx = tuple(int(rng.integers(s)) for s in m0.shape)
        mp, mm = m0.copy(), m0.copy()
        mp[idx] += eps
        mm[idx] -= eps
        dE = (oracle.energies(mesh, mat, mp, term)[key] - oracle.energies(mesh, mat, mm, term)[key]) / (2 * eps)
        want = -dE / M[idx[1:]]
        assert abs(H[idx] - want) <= 1e-7 * max(abs(want), np.abs(H).max())


def test_bulk_dmi_energy_is_quadratic_and_odd_in_d():
    mesh, mat, m0 = _problem(94)
    e = oracle.energies(mesh, mat, m0, DMI)["dmi"]
    g = oracle.gradient(mesh, mat, m0, DMI)
    assert abs(0.5 * np.sum(g * m0) - e) <= 1e-12 * abs(e)      # Euler: E = m . g / 2
    mat.D = -mat.D
    assert abs(oracle.energies(mesh, mat, m0, DMI)["dmi"] + e) <= 1e-12 * abs(e)
    # interfacial and bulk are different operators on the same state
    mat.D = -mat.D
    mat.dmi_type = "interfacial"
    assert abs(oracle.energies(mesh, mat, m0, DMI)["dmi"] - e) > 1e-3 * abs(e)


def test_bulk_dmi_helix_interior_field_is_the_centred_difference():
    """m = (0, cos kx, sin kx) has curl m = -k m; the continuum field is
    H = -(2D / (mu0 Ms)) curl m, and on the grid the derivative becomes the
    centred difference sin(kh)/h exactly (interior nodes)."""
    n = [9, 4, 3]
    h = [2e-9, 2.5e-9, 3e-9]
    mesh = oracle.Mesh(n, h)
    Ms, D = 8e5, 2.5e-3
    mat = oracle.Material(Ms=np.full(mesh.cell_shape, Ms), A=np.full(mesh.cell_shape, 1e-11),
                          alpha=np.zeros(mesh.cell_shape), D=np.full(mesh.cell_shape, D), dmi_type="bulk")
    k = 0.37 / h[0]
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in mesh.node_shape], indexing="ij")
    x = xx * h[0]
    m = np.stack([np.zeros_like(x), np.cos(k * x), np.sin(k * x)])
    H = oracle.heff(mesh, mat, m, DMI)
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    want = (2 * D / (MU0 * Ms)) * np.sin(k * h[0]) / h[0] * m
    assert rel_l2(H[inner], want[inner]) < 1e-12


def _uniform_cubic(mvec, basis="3d"):
    n = (4, 3, 2) if basis == "3d" else (4, 3, 1)
    mesh = oracle.Mesh(n, (2e-9, 2.5e-9, 3e-9), basis=basis)
    cs = mesh.cell_shape
    Ms, Kc = 9e5, 3e5
    th = 0.4
    c1 = np.array([np.cos(th), np.sin(th), 0.0])
    c2 = np.array([-np.sin(th) * np.cos(0.3), np.cos(th) * np.cos(0.3), np.sin(0.3)])
    cubic = np.stack([np.broadcast_to(c.reshape(3, 1, 1, 1), (3,) + cs) for c in (c1, c2)])
    mat = oracle.Material(Ms=np.full(cs, Ms), A=np.full(cs, 1e-11), alpha=np.zeros(cs),
                          Kc=np.full(cs, Kc), cubic=cubic.copy())
    mv = np.asarray(mvec, dtype=np.float64)
    mv = mv / np.linalg.norm(mv)
    m = np.broadcast_to(mv.reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
    axes = (c1, c2, np.cross(c1, c2))
    return mesh, mat, m, mv, axes, Ms, Kc


@pytest.mark.parametrize("basis", ["3d", "film"])
def test_cubic_uniform_state_closed_form(basis):
    """Uniform m and material: H = -(Kc / (mu0 Ms)) df/dm at every node and
    E = Kc V_total f(m), with f = a1^2 a2^2 + a2^2 a3^2 + a3^2 a1^2."""
    mesh, mat, m, mv, axes, Ms, Kc = _uniform_cubic((0.3, -0.5, 0.8), basis)
    a = [float(mv @ c) for c in axes]
    f = a[0] ** 2 * a[1] ** 2 + a[1] ** 2 * a[2] ** 2 + a[2] ** 2 * a[0] ** 2
    df = sum(2 * a[i] * (a[(i + 1) % 3] ** 2 + a[(i + 2) % 3] ** 2) * axes[i] for i in range(3))
    H = oracle.heff(mesh, mat, m, CUBIC)
    want = -(Kc / (MU0 * Ms)) * df
    assert np.abs(H - want.reshape(3, 1, 1, 1)).max() <= 1e-10 * np.abs(want).max()
    e = oracle.energies(mesh, mat, m, CUBIC)["cubic"]
    assert abs(e - Kc * mesh.V * mesh.n_cells * f) <= 1e-12 * abs(e)


def test_cubic_axes_carry_no_torque_and_symmetries():
    # along a cubic axis the field is zero; along a body diagonal it is parallel to m
    for mvec, zero in (("c1", True), ("diag", False)):
        mesh, mat, m, mv, axes, Ms, Kc = _uniform_cubic((1.0, 0.0, 0.0))
        v = axes[0] if mvec == "c1" else (axes[0] + axes[1] + axes[2]) / np.sqrt(3.0)
        m = np.broadcast_to(v.reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
        H = oracle.heff(mesh, mat, m, CUBIC)
        if zero:
            assert np.abs(H).max() <= 1e-12 * Kc / (MU0 * Ms)
        else:
            assert np.abs(np.cross(m, H, axis=0)).max() <= 1e-10 * np.abs(H).max()
    # f is even in m and invariant under permutations of the axes
    rng = np.random.default_rng(3)
    mc = rng.standard_normal((3, 7))
    ax = [synth.random_unit_vectors(1, rng)[:, 0] for _ in range(3)]
    axes = [a.reshape(3, 1) for a in ax]
    f, df = cubic_density_gradient(mc, axes)
    f2, df2 = cubic_density_gradient(-mc, [axes[2], axes[0], axes[1]])
    assert np.allclose(f, f2, rtol=1e-14, atol=0) and np.allclose(df, -df2, rtol=1e-12, atol=1e-15)
