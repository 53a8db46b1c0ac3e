"""Pins of the oracle's discrete adjoint: every transpose is checked against
central finite differences of the forward map it transposes (dot-product
tests), and the field-map gradient against finite differences of the loss."""
import numpy as np
import pytest

import oracle
from oracle.adjoint import (cell_gather, continuous_adjoint, llg_vjp, region_mz2_loss, rhs_vjp,
                            rk4_gradient, rk4_step_adjoint)
from oracle.field import ALL_TERMS, ANISOTROPY, DEMAG, DMI, EXCHANGE, ZEEMAN

from helpers import to_oracle
from paper_2411_11725_amd import synth


def _llg(m, H, alpha_n, gp):
    mxh = np.cross(m, H, axis=0)
    return -gp * mxh - alpha_n * gp * np.cross(m, mxh, axis=0)


def _problem(n=(4, 3, 2), seed=51, dmi=False):
    p = synth.small_random(n, (2e-9, 2.5e-9, 3e-9), seed=seed, dmi=dmi)
    return to_oracle(p)


def test_llg_vjp_against_finite_differences():
    rng = np.random.default_rng(1)
    shape = (3, 2, 3, 4)
    m = rng.standard_normal(shape)
    H = 1e5 * rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    a = rng.uniform(0.01, 1.0, shape[1:])
    gp = 2.211e5 / (1 + a ** 2)
    dm_t, u = llg_vjp(m, H, w, a, gp)
    d = rng.standard_normal(shape)
    eps = 1e-5
    jd = (_llg(m + eps * d, H, a, gp) - _llg(m - eps * d, H, a, gp)) / (2 * eps)
    assert abs(np.sum(jd * w) - np.sum(d * dm_t)) <= 1e-8 * abs(np.sum(d * dm_t))
    dH = 1e4 * rng.standard_normal(shape)
    jh = _llg(m, H + dH, a, gp) - _llg(m, H, a, gp)       # linear in H
    assert abs(np.sum(jh * w) - np.sum(dH * u)) <= 1e-10 * abs(np.sum(dH * u))


@pytest.mark.parametrize("dmi", [False, True])
def test_linear_field_operator_is_self_adjoint_in_the_mass_metric(dmi):
    """M H_lin is the negative Hessian of the quadratic energies: symmetric
    (the DMI element matrices are not, but their energy's Hessian is)."""
    mesh, mat, _ = _problem(dmi=dmi)
    M = oracle.lumped_mass(mesh, mat)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3,) + mesh.node_shape)
    b = rng.standard_normal((3,) + mesh.node_shape)
    lin = EXCHANGE | ANISOTROPY | DEMAG | DMI
    lhs = np.sum(M * oracle.heff(mesh, mat, a, lin) * b)
    rhs = np.sum(a * M * oracle.heff(mesh, mat, b, lin))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("terms,dmi", [(ALL_TERMS, False), (EXCHANGE | DEMAG, False), (ALL_TERMS, True),
                                      (DMI, True)])
def test_rhs_vjp_dot_product(terms, dmi):
    mesh, mat, m = _problem(dmi=dmi)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(m.shape)
    v = rng.standard_normal(m.shape)
    jt, _ = rhs_vjp(mesh, mat, m, 0.0, w, terms)
    eps = 1e-6
    jv = (oracle.llg_rhs(mesh, mat, m + eps * v, 0.0, terms)
          - oracle.llg_rhs(mesh, mat, m - eps * v, 0.0, terms)) / (2 * eps)
    assert abs(np.sum(jv * w) - np.sum(v * jt)) <= 1e-7 * abs(np.sum(v * jt))


def test_rk4_step_adjoint_dot_product():
    mesh, mat, m = _problem(seed=52)
    rng = np.random.default_rng(4)
    lam = rng.standard_normal(m.shape)
    v = rng.standard_normal(m.shape)
    dt = 2e-14
    lam0, _ = rk4_step_adjoint(mesh, mat, m, 0.0, dt, lam, ALL_TERMS)
    eps = 1e-6
    jv = (oracle.rk4_step(mesh, mat, m + eps * v, 0.0, dt)
          - oracle.rk4_step(mesh, mat, m - eps * v, 0.0, dt)) / (2 * eps)
    assert abs(np.sum(jv * lam) - np.sum(v * lam0)) <= 1e-8 * abs(np.sum(v * lam0))


def test_field_map_gradient_against_finite_differences():
    """Magnonic-strip style objective over a short trajectory: the adjoint
    gradient wrt the per-cell field map equals central differences of L."""
    p = synth.magnonic(n=(24, 8, 1))
    mesh, mat, m0 = to_oracle(p)
    nsteps, dt = 12, 5e-14
    region = np.zeros(mesh.node_shape, dtype=bool)
    region[:, 2:6, 14:20] = True
    loss, dloss = region_mz2_loss(mesh, region, nsteps)

    def L(mat_):
        m = m0.copy()
        tot = 0.0
        for k in range(nsteps):
            m = oracle.rk4_step(mesh, mat_, m, k * dt, dt)
            tot += loss(m)
        return tot

    _, dth, _ = rk4_gradient(mesh, mat, m0, dt, nsteps, dloss, ALL_TERMS)
    h = 0.7958  # 1e-3 mT in A/m
    for (j, c3, c2, c1) in [(0, 0, 3, 17), (1, 0, 4, 15), (2, 0, 2, 18), (2, 0, 5, 10)]:
        hp = mat.h_cell.copy()
        hm = mat.h_cell.copy()
        hp[j, c3, c2, c1] += h
        hm[j, c3, c2, c1] -= h
        mp = oracle.Material(**{**mat.__dict__, "h_cell": hp})
        mm = oracle.Material(**{**mat.__dict__, "h_cell": hm})
        fd = (L(mp) - L(mm)) / (2 * h)
        g = dth[j, c3, c2, c1]
        assert abs(g - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(dth).max()), (j, g, fd)


def test_cell_gather_is_transpose_of_field_map():
    """<H_ext(theta), M u'> summed over nodes == <theta, gather(u')>."""
    mesh, mat, _ = _problem()
    rng = np.random.default_rng(5)
    theta = rng.standard_normal((3,) + mesh.cell_shape)
    v = rng.standard_normal((3,) + mesh.node_shape)
    M = oracle.lumped_mass(mesh, mat)
    mat2 = oracle.Material(**{**mat.__dict__, "h_cell": theta, "h_uniform": np.zeros(3)})
    Hz = oracle.heff(mesh, mat2, np.zeros_like(v), ZEEMAN)
    assert abs(np.sum(Hz * M * v) - np.sum(theta * cell_gather(mesh, mat2, v))) <= 1e-12 * np.sum(np.abs(Hz * M * v))


# ---------------------------------------------------------------- continuous
def _linear_final_loss(mesh, seed=2):
    c = np.random.default_rng(seed).standard_normal((3,) + mesh.node_shape)
    return c, (lambda m: float(np.sum(c * m)))


def test_continuous_adjoint_converges_to_the_discrete_adjoint_at_fourth_order():
    """Both are RK4 discretisations of the same gradient: the continuous one
    (Eq. adjoint_system, backwards) differs from the exact gradient of the
    discrete map by O(dt^4), so halving dt divides the gap by ~16; the
    rebuilt initial state converges to m0 at least as fast."""
    mesh, mat, m0 = _problem(n=(5, 4, 2), seed=52)
    c, _ = _linear_final_loss(mesh)
    span = 4e-13
    gaps, back = [], []
    for dt in (4e-14, 2e-14):
        ns = int(round(span / dt))
        lam, th, mT = rk4_gradient(mesh, mat, m0, dt, ns, lambda k, m: np.zeros_like(m), ALL_TERMS,
                                   lam_end=c)
        mb, a0, u0 = continuous_adjoint(mesh, mat, mT, span, dt, ns, c, ALL_TERMS)
        gaps.append(np.linalg.norm(u0 - th) / np.linalg.norm(th) + np.linalg.norm(a0 - lam) / np.linalg.norm(lam))
        back.append(np.abs(mb - m0).max())
    assert gaps[0] < 1e-5 and 10.0 < gaps[0] / gaps[1] < 24.0
    # forward then backward RK4: at least fourth order (the leading terms of
    # the two sweeps partly cancel, so the ratio can exceed 16)
    assert back[0] < 1e-5 and back[0] / back[1] > 10.0


def test_continuous_adjoint_gradient_against_finite_differences():
    """u(0) is the gradient of L = c . m(T) with respect to the field map."""
    mesh, mat, m0 = _problem(n=(4, 3, 2), seed=53)
    c, loss = _linear_final_loss(mesh, seed=3)
    dt, ns = 1e-14, 20

    def L(mat_):
        m = m0.copy()
        for k in range(ns):
            m = oracle.rk4_step(mesh, mat_, m, k * dt, dt)
        return loss(m)

    m = m0.copy()
    for k in range(ns):
        m = oracle.rk4_step(mesh, mat, m, k * dt, dt)
    _, _, u = continuous_adjoint(mesh, mat, m, ns * dt, dt, ns, c, ALL_TERMS)
    h = 0.7958
    for (j, c3, c2, c1) in [(0, 0, 1, 2), (1, 1, 2, 0), (2, 1, 0, 3)]:
        hp = mat.h_cell.copy()
        hm = mat.h_cell.copy()
        hp[j, c3, c2, c1] += h
        hm[j, c3, c2, c1] -= h
        fd = (L(oracle.Material(**{**mat.__dict__, "h_cell": hp}))
              - L(oracle.Material(**{**mat.__dict__, "h_cell": hm}))) / (2 * h)
        assert abs(u[j, c3, c2, c1] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(u).max()), (j, u[j, c3, c2, c1], fd)


def test_macrospin_field_gradient_is_the_closed_form():
    """One cell in a uniform state under a field H z (a macrospin): the polar
    angle follows tan(theta/2) = tan(theta0/2) exp(-alpha gamma' H t), so
    L = <m_z(T)> has dL/dH = sin(theta) * 2 u alpha gamma' T / (1 + u^2),
    u = tan(theta(T)/2); the discrete adjoint's field-map gradient matches it
    up to the O(dt^4) of RK4."""
    mesh = oracle.Mesh((1, 1, 1), (2e-9, 2e-9, 2e-9))
    cs = mesh.cell_shape
    alpha, gamma, H, th0 = 0.5, 2.211e5, 1e5, 1.0
    hc = np.zeros((3,) + cs)
    hc[2] = H
    mat = oracle.Material(Ms=np.full(cs, 8e5), A=np.full(cs, 1e-11), alpha=np.full(cs, alpha),
                          gamma=gamma, h_cell=hc)
    m0 = np.zeros((3,) + mesh.node_shape)
    m0[0], m0[2] = np.sin(th0), np.cos(th0)
    dt, nsteps = 1e-13, 200
    T = dt * nsteps

    def dloss(k, m):
        g = np.zeros_like(m)
        if k == nsteps:
            g[2] = 1.0 / m[2].size
        return g

    _, dth, mT = rk4_gradient(mesh, mat, m0, dt, nsteps, dloss, EXCHANGE | ZEEMAN)
    gp = gamma / (1 + alpha ** 2)
    u = np.tan(th0 / 2) * np.exp(-alpha * gp * H * T)
    theta = 2 * np.arctan(u)
    assert abs(mT[2].mean() - np.cos(theta)) <= 1e-10
    want = np.sin(theta) * 2 * u * alpha * gp * T / (1 + u * u)
    assert abs(dth[2].sum() - want) <= 1e-7 * abs(want)


def test_magnonic_full_size_adjoint_matches_stored_central_differences():
    """The stored full-size record of the inverse-problem workload (256 x 128
    x 1 strip, 4000 RK4 steps; written by tests/golden/make_magnonic_fd.py
    from oracle runs only): at each of the 16 cells the oracle's discrete
    adjoint gradient agrees with the float64 central differences of its own
    objective, |g - g_fd| / max(|g|, 1e-3 max|g|) <= 5e-6, and the
    differences were taken with h = 1e-3 mT."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "magnonic_fd.txt")
    rows, header = [], ""
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                header += line
            elif line[0].isdigit():
                rows.append([float(v) for v in line.split()])
    assert "h = 1e-3 mT = 7.9577471546e-01 A/m" in header
    assert len(rows) == 16 and all(len(r) == 8 for r in rows)
    h = 1e-6 / (4e-7 * np.pi)
    fd = np.array([r[4] for r in rows])
    # the stored difference quotient is the stored pair of objective values
    assert np.allclose(fd, np.array([(r[5] - r[6]) / (2 * h) for r in rows]), rtol=1e-9, atol=0)
    adj = np.array([r[7] for r in rows])
    floor = np.maximum(np.abs(adj), 1e-3 * np.abs(adj).max())
    assert (np.abs(adj - fd) / floor).max() <= 5e-6
