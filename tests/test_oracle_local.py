"""Pins of the oracle's local terms (exchange, anisotropy, Zeeman, mass).

Each test checks the oracle against something other than itself: a value the
paper prints, a closed form of the continuous problem, or an invariant.
"""
import os

import numpy as np
import pytest

import oracle
from oracle.field import ANISOTROPY, DEMAG, EXCHANGE, ZEEMAN
from oracle.mesh import CORNERS

from helpers import rel_l2, to_oracle
from paper_2411_11725_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MU0 = 4e-7 * np.pi


def _problem(n=(5, 4, 3), h=(2e-9, 3e-9, 2.5e-9), seed=3, **kw):
    return to_oracle(synth.small_random(n, h, seed=seed, **kw))


def test_lst2_exchange_diagonal_coefficient():
    """Sec. 5.1, Lst. form_code: the printed coefficient (2/9, to 15 digits)
    of a node's own value in the generated exchange element, times the sum
    of h_i h_j / h_k over the axis permutations."""
    with open(os.path.join(GOLDEN, "lst2_exchange_diagonal.txt")) as fh:
        coef = [float(l.split()[1]) for l in fh if l.startswith("coefficient")][0]
    rng = np.random.default_rng(0)
    for _ in range(5):
        h = tuple(rng.uniform(0.5, 3.0, 3))
        mesh = oracle.Mesh((1, 1, 1), h)
        mat = oracle.Material(Ms=np.ones((1, 1, 1)), A=np.ones((1, 1, 1)),
                              alpha=np.zeros((1, 1, 1)))
        m = np.zeros((3,) + mesh.node_shape)
        m[0, 0, 0, 0] = 1.0
        g = oracle.gradient(mesh, mat, m, EXCHANGE)
        want = coef * (h[0] * h[1] / h[2] + h[0] * h[2] / h[1] + h[1] * h[2] / h[0])
        assert abs(g[0, 0, 0, 0] - want) <= 1e-14 * want


def test_element_matrices_match_gauss_quadrature():
    """Closed-form Kronecker factors == 2-point Gauss quadrature of Eq. nodal_basis."""
    mesh = oracle.Mesh((1, 1, 1), (1.3, 0.7, 2.1))
    K, M = mesh.element_matrices()
    Kq, Mq = mesh.element_matrices_quadrature()
    assert np.allclose(K, Kq, rtol=0, atol=1e-13)
    assert np.allclose(M, Mq, rtol=0, atol=1e-13)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-13)
    assert abs(M.sum() - mesh.V) < 1e-13
    assert np.allclose(M.sum(axis=1), mesh.V / 8.0, atol=1e-14)


def test_cubic_interior_stencil_weights():
    """Assembled exchange operator on cubic cells: centre 8/3 h, faces 0,
    edges -1/6 h, corners -1/12 h (times 2A)."""
    h = 1.7
    mesh = oracle.Mesh((4, 4, 4), (h, h, h))
    mat = oracle.Material(Ms=np.ones(mesh.cell_shape), A=np.ones(mesh.cell_shape),
                          alpha=np.zeros(mesh.cell_shape))
    m = np.zeros((3,) + mesh.node_shape)
    m[1, 2, 2, 2] = 1.0
    g = oracle.gradient(mesh, mat, m, EXCHANGE)[1]
    for d3 in (-1, 0, 1):
        for d2 in (-1, 0, 1):
            for d1 in (-1, 0, 1):
                k = abs(d1) + abs(d2) + abs(d3)
                want = 2.0 * h * {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[k]
                assert abs(g[2 + d3, 2 + d2, 2 + d1] - want) < 1e-12
    assert abs(g.sum()) < 1e-12  # rows sum to zero


def test_uniform_m_has_no_exchange():
    mesh, mat, _ = _problem()
    m = np.ones((3,) + mesh.node_shape) * np.array([0.6, -0.8, 0.0]).reshape(3, 1, 1, 1)
    H = oracle.heff(mesh, mat, m, EXCHANGE)
    assert np.abs(H).max() < 1e-6  # vs ~1e7 A/m scale of the term
    assert abs(oracle.energies(mesh, mat, m, EXCHANGE)["exchange"]) < 1e-30


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_spin_spiral_is_three_point_laplacian(axis):
    """m = (cos kx, sin kx, 0): H_ex = -(2A/(mu0 Ms)) 2(1 - cos k h)/h^2 m at every
    node, the free surfaces acting as mirrored ghosts (natural BC, Eq.
    exchange_variation)."""
    n = [6, 5, 4]
    h = [2e-9, 2.5e-9, 3e-9]
    mesh = oracle.Mesh(n, h)
    A, Ms = 1.3e-11, 8e5
    mat = oracle.Material(Ms=np.full(mesh.cell_shape, Ms), A=np.full(mesh.cell_shape, A),
                          alpha=np.zeros(mesh.cell_shape))
    k = 0.37 / h[axis]
    coords = np.meshgrid(np.arange(n[2] + 1), np.arange(n[1] + 1), np.arange(n[0] + 1),
                         indexing="ij")
    x = coords[2 - axis] * h[axis]
    m = np.stack([np.cos(k * x), np.sin(k * x), np.zeros_like(x)])
    H = oracle.heff(mesh, mat, m, EXCHANGE)
    lap = 2.0 * (1.0 - np.cos(k * h[axis])) / h[axis] ** 2
    want = -(2 * A / (MU0 * Ms)) * lap * m
    idx = [slice(None)] * 4
    idx[3 - axis] = slice(1, -1)  # interior along the spiral axis
    assert rel_l2(H[tuple(idx)], want[tuple(idx)]) < 1e-12
    # free surface: ghost m_{-1} = m_{1}  =>  2 (m_0 - m_1)/h^2
    s0 = [slice(None)] * 4
    s1 = [slice(None)] * 4
    s0[3 - axis] = 0
    s1[3 - axis] = 1
    want0 = -(2 * A / (MU0 * Ms)) * 2.0 * (m[tuple(s0)] - m[tuple(s1)]) / h[axis] ** 2
    assert rel_l2(H[tuple(s0)], want0) < 1e-12


def test_uniform_anisotropy_and_zeeman_closed_forms():
    n = (4, 3, 2)
    mesh = oracle.Mesh(n, (2e-9, 3e-9, 4e-9))
    cs = mesh.cell_shape
    Ms, K = 7e5, 3e5
    e = np.array([1.0, 2.0, 2.0]) / 3.0
    Hx = np.array([1e4, -3e4, 2e4])
    mat = oracle.Material(Ms=np.full(cs, Ms), A=np.full(cs, 1e-11), alpha=np.zeros(cs),
                          Ku=np.full(cs, K), easy=np.broadcast_to(e.reshape(3, 1, 1, 1), (3,) + cs).copy(),
                          h_uniform=Hx)
    mv = np.array([0.48, -0.6, 0.64])
    m = np.broadcast_to(mv.reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
    Ha = oracle.heff(mesh, mat, m, ANISOTROPY)
    want = (2 * K / (MU0 * Ms)) * (mv @ e) * e
    assert np.allclose(Ha, want.reshape(3, 1, 1, 1), rtol=1e-13, atol=0)
    Hz = oracle.heff(mesh, mat, m, ZEEMAN)
    assert np.allclose(Hz, Hx.reshape(3, 1, 1, 1), rtol=1e-13, atol=0)
    Vt = mesh.V * mesh.n_cells
    E = oracle.energies(mesh, mat, m, ANISOTROPY | ZEEMAN)
    assert abs(E["anisotropy"] - (-K * Vt * (mv @ e) ** 2)) < 1e-12 * K * Vt
    assert abs(E["zeeman"] - (-MU0 * Ms * Vt * (mv @ Hx))) < 1e-12 * abs(MU0 * Ms * Vt * (mv @ Hx))


def test_drive_field_time_dependence():
    p = synth.magnonic(n=(24, 8, 1))
    mesh, mat, m = to_oracle(p)
    t = 0.3e-10
    H = oracle.external_cell_field(mesh, mat, t)
    s = np.sin(2 * np.pi * 10e9 * t)
    assert np.allclose(H[1, :, :, 16:20], p["drive_amp"][1] * s, rtol=1e-12)
    assert np.all(H[1, :, :, :16] == 0.0)


def test_lumped_mass_sums_to_total_moment():
    mesh, mat, _ = _problem()
    M = oracle.lumped_mass(mesh, mat)
    assert abs(M.sum() - MU0 * mesh.V * mat.Ms.sum()) < 1e-12 * M.sum()
    # corner node belongs to one cell only
    assert abs(M[0, 0, 0] - MU0 * mat.Ms[0, 0, 0] * mesh.V / 8) < 1e-25


@pytest.mark.parametrize("term", [EXCHANGE, ANISOTROPY, ZEEMAN, DEMAG])
def test_field_is_minus_energy_gradient_over_mass(term):
    """Eq. heff with Eq. mass_lumping: dE/dm_n = -M_n H_n, checked by central
    differences of the energy functional along a random direction."""
    mesh, mat, m = _problem(n=(4, 3, 3), seed=11)
    H = oracle.heff(mesh, mat, m, term)
    M = oracle.lumped_mass(mesh, mat)
    rng = np.random.default_rng(5)
    d = rng.standard_normal(m.shape)
    eps = 1e-4
    Ep = oracle.energies(mesh, mat, m + eps * d, term)["total"]
    Em = oracle.energies(mesh, mat, m - eps * d, term)["total"]
    fd = (Ep - Em) / (2 * eps)
    an = float(np.sum(-M * H * d))
    assert abs(fd - an) <= 1e-8 * abs(an)


def test_quadratic_energy_euler_identity():
    """E is homogeneous of degree 2 in m for exchange, anisotropy and demag,
    and of degree 1 for Zeeman: E = -(mu0/2) sum M H.m  resp.  -sum M H.m."""
    mesh, mat, m = _problem(n=(5, 4, 2), seed=13)
    M = oracle.lumped_mass(mesh, mat)
    for term in (EXCHANGE, ANISOTROPY, DEMAG):
        H = oracle.heff(mesh, mat, m, term)
        E = oracle.energies(mesh, mat, m, term)["total"]
        assert abs(E - (-0.5 * np.sum(M * H * m))) <= 1e-11 * abs(E)
    H = oracle.heff(mesh, mat, m, ZEEMAN)
    E = oracle.energies(mesh, mat, m, ZEEMAN)["total"]
    assert abs(E - (-np.sum(M * H * m))) <= 1e-11 * abs(E)


def test_exchange_jump_two_phase_interface():
    """Two materials A1 | A2 along x with a profile that is piecewise linear with
    A1 dm/dx = A2 dm/dx across the interface (Eq. exchange_jump): interior
    nodes, including the interface node, feel no exchange field."""
    n = (8, 2, 2)
    h = (1e-9, 1e-9, 1e-9)
    mesh = oracle.Mesh(n, h)
    A = np.full(mesh.cell_shape, 1e-11)
    A[:, :, 4:] = 3e-11
    mat = oracle.Material(Ms=np.full(mesh.cell_shape, 8e5), A=A, alpha=np.zeros(mesh.cell_shape))
    x = np.arange(n[0] + 1)
    slope1 = 0.03
    slope2 = slope1 * 1e-11 / 3e-11
    prof = np.where(x <= 4, slope1 * x, 4 * slope1 + slope2 * (x - 4))
    m = np.zeros((3,) + mesh.node_shape)
    m[1] = prof[None, None, :]
    H = oracle.heff(mesh, mat, m, EXCHANGE)
    assert np.abs(H[1, :, :, 1:-1]).max() < 1e-9 * np.abs(H[1]).max() + 1e-6
