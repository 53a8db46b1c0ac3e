"""Pins of the oracle's thin-film basis (bilinear in-plane, constant along z;
Sec. 3.3, low-dimensional geometries).

Each test checks the film oracle against something other than itself: its
element matrices against Gauss quadrature of the 2D reference functions, the
full 3D discretisation of a single cell layer (the film basis function of a
node is the sum of the two 3D functions above each other, so for m constant
along z the two must give the same field and energies), and the closed form
of an in-plane spin spiral.
"""
import numpy as np
import pytest

import oracle
from oracle.field import ALL_TERMS, ANISOTROPY, DEMAG, DMI, EXCHANGE, ZEEMAN

from helpers import rel_l2, to_oracle
from paper_2411_11725_amd import synth

MU0 = 4e-7 * np.pi


def _film(n=(7, 5, 1), h=(3.9e-9, 3.1e-9, 2.5e-9), seed=31, **kw):
    p = synth.small_random(n, h, seed=seed, **kw)
    mesh3, mat, _ = to_oracle(p)
    film = oracle.Mesh(p["n"], p["h"], basis="film")
    rng = np.random.default_rng(seed + 1)
    m = rng.normal(size=(3,) + film.node_shape)
    m /= np.linalg.norm(m, axis=0)
    return film, mesh3, mat, m


def test_film_element_matrices_match_gauss_quadrature():
    mesh = oracle.Mesh((1, 1, 1), (1.3, 0.7, 2.1), basis="film")
    K, M = mesh.element_matrices()
    Kq, Mq = mesh.element_matrices_quadrature()
    assert K.shape == (4, 4)
    assert np.allclose(K, Kq, rtol=0, atol=1e-13)
    assert np.allclose(M, Mq, rtol=0, atol=1e-13)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-13)
    assert abs(M.sum() - mesh.V) < 1e-13
    assert np.allclose(M.sum(axis=1), mesh.V / 4.0, atol=1e-14)


@pytest.mark.parametrize("terms", [EXCHANGE, ANISOTROPY, ZEEMAN, DEMAG, DMI, ALL_TERMS])
def test_film_field_equals_3d_field_of_z_uniform_m(terms):
    film, mesh3, mat, m = _film(ku_range=(-5e5, 5e5), dmi=True)
    m3 = np.concatenate([m, m], axis=1)          # both node layers of the cell layer
    H2 = oracle.heff(film, mat, m, terms, t=1e-11)
    H3 = oracle.heff(mesh3, mat, m3, terms, t=1e-11)
    assert rel_l2(H2, H3[:, 0:1]) < 1e-12
    assert rel_l2(H2, H3[:, 1:2]) < 1e-12
    e2 = oracle.energies(film, mat, m, terms, t=1e-11)
    e3 = oracle.energies(mesh3, mat, m3, terms, t=1e-11)
    for k in ("exchange", "demag", "anisotropy", "zeeman", "dmi", "total"):
        assert abs(e2[k] - e3[k]) <= 1e-12 * max(abs(e3["total"]), abs(e3[k]), 1e-30)


def test_film_lumped_mass_is_the_two_layers_together():
    film, mesh3, mat, _ = _film()
    M2 = oracle.lumped_mass(film, mat)
    M3 = oracle.lumped_mass(mesh3, mat)
    assert np.allclose(M2[0], M3[0] + M3[1], rtol=1e-14, atol=0)
    assert abs(M2.sum() - MU0 * np.sum(mat.Ms) * film.V) < 1e-12 * M2.sum()


@pytest.mark.parametrize("axis", [0, 1])
def test_film_spin_spiral_is_three_point_laplacian(axis):
    """In-plane spiral m = (cos kx, sin kx, 0): interior nodes carry the 1D
    three-point Laplacian, the free edges the mirrored-ghost boundary value."""
    n = [6, 5, 1]
    h = [2e-9, 2.5e-9, 3e-9]
    mesh = oracle.Mesh(n, h, basis="film")
    A, Ms = 1.3e-11, 8e5
    mat = oracle.Material(Ms=np.full(mesh.cell_shape, Ms), A=np.full(mesh.cell_shape, A),
                          alpha=np.zeros(mesh.cell_shape))
    k = 0.37 / h[axis]
    yy, xx = np.meshgrid(np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
    x = (xx if axis == 0 else yy)[None] * h[axis]
    m = np.stack([np.cos(k * x), np.sin(k * x), np.zeros_like(x)])
    H = oracle.heff(mesh, mat, m, EXCHANGE)
    lap = 2.0 * (1.0 - np.cos(k * h[axis])) / h[axis] ** 2
    want = -(2 * A / (MU0 * Ms)) * lap * m
    idx = [slice(None)] * 4
    idx[3 - axis] = slice(1, -1)
    assert rel_l2(H[tuple(idx)], want[tuple(idx)]) < 1e-12
    s0 = [slice(None)] * 4
    s1 = [slice(None)] * 4
    s0[3 - axis] = 0
    s1[3 - axis] = 1
    want0 = -(2 * A / (MU0 * Ms)) * 2.0 * (m[tuple(s0)] - m[tuple(s1)]) / h[axis] ** 2
    assert rel_l2(H[tuple(s0)], want0) < 1e-12


def test_film_uniform_m_has_no_exchange_and_rhs_keeps_norm():
    film, _, mat, m = _film()
    u = np.ones((3,) + film.node_shape) / np.sqrt(3.0)
    assert np.abs(oracle.heff(film, mat, u, EXCHANGE)).max() < 1e-6
    f = oracle.llg_rhs(film, mat, m)
    assert np.abs(np.sum(f * m, axis=0)).max() < 1e-9 * np.abs(f).max()


def test_film_basis_needs_one_cell_layer():
    with pytest.raises(ValueError):
        oracle.Mesh((4, 4, 2), (1e-9,) * 3, basis="film")
