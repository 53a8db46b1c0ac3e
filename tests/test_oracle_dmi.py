"""Pins of the oracle's interfacial antisymmetric exchange (DMI, interface
normal along z):  E = sum_c D_c int_c [m_z div m - (m . grad) m_z].

The element matrices are checked against Gauss quadrature of the reference
functions, the field against finite differences of the energy, and an
interior cycloid against the centred difference of the continuum field
H = (2D / (mu0 Ms)) (d_x m_z, d_y m_z, -d_x m_x - d_y m_y).
"""
import numpy as np
import pytest

import oracle
from oracle.field import DMI

from helpers import rel_l2, to_oracle
from paper_2411_11725_amd import synth

MU0 = 4e-7 * np.pi


@pytest.mark.parametrize("basis", ["3d", "film"])
def test_dmi_element_matrices_match_gauss_quadrature(basis):
    mesh = oracle.Mesh((1, 1, 1), (1.3e-9, 0.7e-9, 2.1e-9), basis=basis)
    G = mesh.element_dmi()
    Gq = mesh.element_dmi_quadrature()
    assert np.allclose(G, Gq, rtol=0, atol=1e-12 * np.abs(G).max())
    # sum over a of G_k[a, b] = int d_k phi_b: the jump of phi_b across the
    # cell along k times the mean of its other factors, +-(face area)/4 (3D)
    # or /2 (film, constant along z)
    area = [mesh.V / mesh.h[0], mesh.V / mesh.h[1]]
    for k in range(2):
        col = G[k].sum(axis=0)
        want = np.array([(1.0 if b[k] == 1 else -1.0) * area[k] for b in mesh.corners])
        want /= 4.0 if basis == "3d" else 2.0
        assert np.allclose(col, want, rtol=1e-12, atol=0)


def _dmi_problem(seed=91, n=(5, 4, 3)):
    p = synth.small_random(n, (2e-9, 2.5e-9, 3e-9), seed=seed)
    mesh, mat, m0 = to_oracle(p)
    mat.D = np.random.default_rng(seed).uniform(-3e-3, 3e-3, size=mesh.cell_shape)
    return mesh, mat, m0


def test_dmi_field_is_minus_energy_gradient_over_mass():
    mesh, mat, m0 = _dmi_problem()
    H = oracle.heff(mesh, mat, m0, DMI)
    M = oracle.lumped_mass(mesh, mat)
    rng = np.random.default_rng(5)
    eps = 1e-6
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in m0.shape)
        mp, mm = m0.copy(), m0.copy()
        mp[idx] += eps
        mm[idx] -= eps
        dE = (oracle.energies(mesh, mat, mp, DMI)["dmi"] - oracle.energies(mesh, mat, mm, DMI)["dmi"]) / (2 * eps)
        want = -dE / M[idx[1:]]
        assert abs(H[idx] - want) <= 1e-7 * max(abs(want), np.abs(H).max())


def test_dmi_energy_is_quadratic_and_antisymmetric_in_d():
    mesh, mat, m0 = _dmi_problem(seed=92)
    e = oracle.energies(mesh, mat, m0, DMI)["dmi"]
    g = oracle.gradient(mesh, mat, m0, DMI)
    assert abs(0.5 * np.sum(g * m0) - e) <= 1e-12 * abs(e)      # Euler: E = m . g / 2
    mat.D = -mat.D
    assert abs(oracle.energies(mesh, mat, m0, DMI)["dmi"] + e) <= 1e-12 * abs(e)


@pytest.mark.parametrize("basis", ["3d", "film"])
def test_dmi_cycloid_interior_field_is_the_centred_difference(basis):
    n = [8, 5, 3] if basis == "3d" else [8, 5, 1]
    h = [2e-9, 2.5e-9, 3e-9]
    mesh = oracle.Mesh(n, h, basis=basis)
    Ms, D = 8e5, 2.5e-3
    mat = oracle.Material(Ms=np.full(mesh.cell_shape, Ms), A=np.full(mesh.cell_shape, 1e-11),
                          alpha=np.zeros(mesh.cell_shape), D=np.full(mesh.cell_shape, D))
    k = 0.41 / h[0]
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in mesh.node_shape], indexing="ij")
    x = xx * h[0]
    m = np.stack([np.sin(k * x), np.zeros_like(x), np.cos(k * x)])
    H = oracle.heff(mesh, mat, m, DMI)
    c = 2 * D / (MU0 * Ms)
    # interior along x and y (the DMI boundary condition acts at the edges)
    inner = (slice(None), slice(None), slice(1, -1), slice(1, -1))
    # centred differences of m_z and m_x along x
    dz = (np.cos(k * (x + h[0])) - np.cos(k * (x - h[0]))) / (2 * h[0])
    dx = (np.sin(k * (x + h[0])) - np.sin(k * (x - h[0]))) / (2 * h[0])
    want = np.stack([c * dz, np.zeros_like(x), -c * dx])
    assert rel_l2(H[inner], want[inner]) < 1e-12
