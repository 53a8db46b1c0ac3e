"""Pins of the oracle's LLG right-hand side and integrators (Eq. llg, Sec. 5.3)."""
import numpy as np
import pytest

import oracle
from oracle.llg import DP45

from helpers import to_oracle
from paper_2411_11725_amd import synth


def _macrospin(alpha, H=1e5, theta0=np.pi / 3, phi0=0.3, A=1.3e-11):
    """One cubic cell with uniform m in a field along z: exchange vanishes and
    the cube's self demag field is parallel to m, so the nodes follow the
    macrospin LLG exactly."""
    mesh = oracle.Mesh((1, 1, 1), (3e-9, 3e-9, 3e-9))
    cs = mesh.cell_shape
    mat = oracle.Material(Ms=np.full(cs, 8e5), A=np.full(cs, A),
                          alpha=np.full(cs, alpha), gamma=2.211e5,
                          h_uniform=np.array([0.0, 0.0, H]))
    m0 = np.array([np.sin(theta0) * np.cos(phi0), np.sin(theta0) * np.sin(phi0), np.cos(theta0)])
    m = np.broadcast_to(m0.reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
    return mesh, mat, m


def _closed_form(alpha, t, H=1e5, theta0=np.pi / 3, phi0=0.3, gamma=2.211e5):
    gp = gamma / (1 + alpha ** 2)
    phi = phi0 + gp * H * t
    theta = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * gp * H * t))
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


@pytest.mark.parametrize("alpha", [0.0, 0.1, 1.0])
def test_macrospin_precession_and_damping(alpha):
    """alpha = 0: Larmor precession at gamma H; alpha > 0: the closed form
    phi = phi0 + g' H t, tan(theta/2) = tan(theta0/2) exp(-alpha g' H t)."""
    mesh, mat, m = _macrospin(alpha)
    T, n = 1e-10, 1000
    mT, _ = oracle.rk4_solve(mesh, mat, m, T / n, n)
    want = _closed_form(alpha, T)
    assert np.abs(mT - want.reshape(3, 1, 1, 1)).max() < 1e-10


def test_rk4_is_fourth_order():
    # A = 0: steps this long are beyond the exchange stability limit, which
    # would amplify rounding-level non-uniformity of the 8 nodes
    mesh, mat, m = _macrospin(0.1, A=0.0)
    T = 2e-10
    errs = []
    for n in (100, 200):
        mT, _ = oracle.rk4_solve(mesh, mat, m, T / n, n)
        errs.append(np.abs(mT[:, 0, 0, 0] - _closed_form(0.1, T)).max())
    assert 14.0 < errs[0] / errs[1] < 18.0


def _tree_conditions(b, A, c):
    """Butcher order conditions up to order 5 (the 17 rooted trees)."""
    Ac = A @ c
    Ac2 = A @ c ** 2
    Ac3 = A @ c ** 3
    AAc = A @ Ac
    return [
        (b.sum(), 1.0), (b @ c, 1 / 2),
        (b @ c ** 2, 1 / 3), (b @ Ac, 1 / 6),
        (b @ c ** 3, 1 / 4), (b @ (c * Ac), 1 / 8), (b @ Ac2, 1 / 12), (b @ AAc, 1 / 24),
        (b @ c ** 4, 1 / 5), (b @ (c ** 2 * Ac), 1 / 10), (b @ (c * Ac2), 1 / 15),
        (b @ (c * AAc), 1 / 30), (b @ Ac ** 2, 1 / 20), (b @ Ac3, 1 / 20),
        (b @ (A @ (c * Ac)), 1 / 40), (b @ (A @ Ac2), 1 / 60), (b @ (A @ AAc), 1 / 120),
    ]


def test_dormand_prince_order_conditions():
    A = np.zeros((7, 7))
    for i, row in enumerate(DP45.a):
        A[i, :len(row)] = row
    c = DP45.c
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)
    cond5 = _tree_conditions(DP45.b, A, c)
    for got, want in cond5:
        assert abs(got - want) < 1e-14
    cond = _tree_conditions(DP45.bstar, A, c)
    for got, want in cond[:8]:          # embedded pair: order 4
        assert abs(got - want) < 1e-14
    # ... and not order 5, so the error estimate is non-trivial
    assert max(abs(g - w) for g, w in cond[8:]) > 1e-6
    assert np.allclose(A[6], DP45.b)    # first same as last


def test_dp45_fixed_steps_are_fifth_order():
    mesh, mat, m = _macrospin(0.1, A=0.0)
    T = 2e-10
    errs = []
    for n in (20, 40):
        dt = T / n
        mT = oracle.dp45_replay(mesh, mat, m, [(k * dt, dt) for k in range(n)])
        errs.append(np.abs(mT[:, 0, 0, 0] - _closed_form(0.1, T)).max())
    assert 26.0 < errs[0] / errs[1] < 38.0


def test_dp45_adaptive_meets_tolerance():
    mesh, mat, m = _macrospin(0.2, A=0.0)
    T = 3e-10
    mT, log = oracle.dp45_solve(mesh, mat, m, 0.0, T, 1e-13, rtol=1e-8, atol=1e-8)
    acc = [x for x in log if x[2]]
    assert abs(sum(x[1] for x in acc) - T) < 1e-22
    assert np.abs(mT[:, 0, 0, 0] - _closed_form(0.2, T)).max() < 1e-6
    assert len(acc) < 200


def test_rhs_conserves_norm_and_dissipates_energy():
    """m . f = 0 node by node; dE/dt = -sum_n M_n alpha_n g'_n |m x H|^2 <= 0."""
    p = synth.small_random((4, 3, 3), (2e-9, 2.5e-9, 3e-9), seed=31)
    mesh, mat, m = to_oracle(p)
    f = oracle.llg_rhs(mesh, mat, m)
    assert np.abs(np.sum(m * f, axis=0)).max() <= 1e-12 * np.abs(f).max()
    H = oracle.heff(mesh, mat, m)
    M = oracle.lumped_mass(mesh, mat)
    a = oracle.nodal_alpha(mesh, mat)
    gp = mat.gamma / (1 + a ** 2)
    want = -np.sum(M * a * gp * np.sum(np.cross(m, H, axis=0) ** 2, axis=0))
    eps = 1e-16
    Ep = oracle.energies(mesh, mat, m + eps * f)["total"]
    Em = oracle.energies(mesh, mat, m - eps * f)["total"]
    assert want < 0
    assert abs((Ep - Em) / (2 * eps) - want) <= 1e-6 * abs(want)


def test_undamped_rk4_conserves_energy_and_norm():
    p = synth.small_random((4, 4, 2), (2e-9, 2e-9, 2e-9), seed=32, field=False)
    mesh, mat, m = to_oracle(p)
    mat.alpha[...] = 0.0
    E0 = oracle.energies(mesh, mat, m)["total"]
    mT, _ = oracle.rk4_solve(mesh, mat, m, 2e-15, 200)
    E1 = oracle.energies(mesh, mat, mT)["total"]
    assert abs(E1 - E0) < 1e-6 * abs(E0)
    # |m_n| is kept node by node (m0 is float32-rounded, so compare with it)
    assert np.abs(np.linalg.norm(mT, axis=0) - np.linalg.norm(m, axis=0)).max() < 1e-10
