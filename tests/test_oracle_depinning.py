"""Pins of the oracle's two-phase depinning (the second validation of
Sec. "Validation", Tab. sp_dw, on chains of our own parameters).

The closed form is checked against a fine-grid relaxation of the continuum
energy written here from scratch (finite differences on a 0.05 nm grid,
scipy's L-BFGS), including the interface angle of the pinned wall; the
oracle's discrete threshold against the closed form as the cells shrink
(second-order convergence, and the K-only case, whose threshold does not
depend on the cell size); the stored fixture against a fresh oracle run;
and the restriction to states uniform across the chain's section against the
unrestricted LLG dynamics."""
import os

import numpy as np
import pytest
from scipy.optimize import minimize

from helpers import to_oracle
from oracle import depinning as dp
from paper_2411_11725_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depinning_fields.txt")


def _continuum_relax(p1, p2, b, d=0.05e-9, soft_len=60e-9, hard_len=30e-9, theta=None):
    """Minimise sum_links A (dtheta)^2 / d + sum_nodes w [K sin^2 + b Ms cos]
    (energy per area of the 1D wall, field -H z) on a grid of spacing d with
    the phase boundary on a node."""
    (A1, K1, M1), (A2, K2, M2) = p1, p2
    n_s, n_h = int(round(soft_len / d)), int(round(hard_len / d))
    N = n_s + n_h
    A = np.where(np.arange(N) < n_s, A1, A2)                 # per link
    wK = np.zeros(N + 1)
    wM = np.zeros(N + 1)
    for i, (K, M) in enumerate(zip(np.where(np.arange(N) < n_s, K1, K2), np.where(np.arange(N) < n_s, M1, M2))):
        wK[i] += 0.5 * d * K
        wK[i + 1] += 0.5 * d * K
        wM[i] += 0.5 * d * M
        wM[i + 1] += 0.5 * d * M
    if theta is None:
        w = np.sqrt(A1 / K1)
        x = np.arange(N + 1) * d
        theta = 2.0 * np.arctan(np.exp(-(x - (n_s * d - 2.0 * w)) / w))
    scale = 1.0 / (K2 * (soft_len + hard_len))

    def f(th):
        dt = np.diff(th)
        e = np.sum(A * dt * dt) / d + np.sum(wK * np.sin(th) ** 2 + b * wM * np.cos(th))
        g = np.zeros_like(th)
        g[:-1] -= 2 * A * dt / d
        g[1:] += 2 * A * dt / d
        g += wK * 2 * np.sin(th) * np.cos(th) - b * wM * np.sin(th)
        return e * scale, g * scale

    res = minimize(f, theta, jac=True, method="L-BFGS-B",
                   options={"gtol": 1e-13, "ftol": 0.0, "maxiter": 500000, "maxcor": 30})
    return res.x, n_s


@pytest.mark.parametrize("case", ["A/K/Ms", "A/Ms", "K"])
def test_closed_form_is_the_continuum_threshold(case):
    p1, p2 = synth.depinning_phases(case)
    bc = dp.closed_form_field(p1, p2)
    th, n_s = _continuum_relax(p1, p2, 0.7 * bc)
    assert not dp.depinned(th, n_s)
    # interface angle of the pinned wall from the first integrals
    assert abs(th[n_s] - dp.interface_angle(p1, p2, 0.7 * bc)) <= 5e-3
    th98, _ = _continuum_relax(p1, p2, 0.98 * bc, theta=th)
    assert not dp.depinned(th98, n_s)
    th102, _ = _continuum_relax(p1, p2, 1.02 * bc, theta=th98)
    assert dp.depinned(th102, n_s)


def test_closed_form_limits():
    """No jump, no pinning; equal A and Ms: (K2 - K1) / (2 Ms); the interface
    condition has a double root at the closed-form field."""
    hard = (1e-11, 1e6, 1e6)
    assert dp.closed_form_field(hard, hard) == 0.0
    assert dp.closed_form_field((1e-11, 2e5, 1e6), hard) == pytest.approx(0.4, rel=1e-14)
    for case in synth.DEPIN_CASES:
        p1, p2 = synth.depinning_phases(case)
        bc = dp.closed_form_field(p1, p2)
        dp.interface_angle(p1, p2, bc * (1 - 1e-9))
        with pytest.raises(ValueError):
            dp.interface_angle(p1, p2, bc * (1 + 1e-6))


def _discrete(case, hx):
    p = synth.two_phase_chain(case, hx=hx)
    mesh, mat, m0 = to_oracle(p)
    bc = dp.closed_form_field(*synth.depinning_phases(case))
    lo, hi = dp.discrete_depinning_field(mesh, mat, m0, p["n_soft"], 0.5 * bc, 1.5 * bc, rel_tol=1e-3)
    return 0.5 * (lo + hi), bc


def test_discrete_threshold_converges_at_second_order():
    b1, bc = _discrete("A/K/Ms", 1e-9)
    b2, _ = _discrete("A/K/Ms", 0.5e-9)
    e1, e2 = (b1 - bc) / bc, (b2 - bc) / bc
    assert 0 < e2 < e1 < 0.05
    assert 3.0 < e1 / e2 < 6.5


def test_k_jump_threshold_does_not_depend_on_the_cell_size():
    b, bc = _discrete("K", 2e-9)
    assert abs(b - bc) <= 2e-3 * bc


def test_fixture_matches_a_fresh_oracle_run():
    rows = [ln.split() for ln in open(GOLDEN) if not ln.startswith("#")]
    got = {(r[0], float(r[1])): tuple(map(float, r[2:])) for r in rows}
    assert {c for c, _ in got} == set(synth.DEPIN_CASES)
    bc, lo, hi = got[("K/Ms", 1e-9)]
    b, bc2 = _discrete("K/Ms", 1e-9)
    assert bc == pytest.approx(bc2, rel=1e-6)
    assert lo <= b <= hi


@pytest.mark.parametrize("hyz,grows", [(1e-9, False), (4e-9, True)])
def test_uniform_section_is_stable_only_for_cubic_cells(hyz, grows):
    """The discrete threshold minimises over states uniform across the chain's
    section.  With cubic cells a perturbation of the pinned wall decays under
    the LLG dynamics (so that restriction holds); with cells four times
    longer across, a checkerboard of the in-plane part across the section
    lowers the energy of the narrow wall and grows."""
    import dataclasses

    import oracle
    p = synth.two_phase_chain("A/Ms", hx=1e-9, hyz=hyz, soft_len=20e-9, hard_len=10e-9)
    mesh, mat, m0 = to_oracle(p)
    matb = dataclasses.replace(mat, h_uniform=np.array([0.0, 0.0, -0.29 / oracle.MU0]))
    rng = np.random.default_rng(0)
    m = m0 + 1e-3 * rng.standard_normal(m0.shape)
    m /= np.linalg.norm(m, axis=0)
    for k in range(1500):
        m = oracle.rk4_step(mesh, matb, m, k * 1e-13, 1e-13, dp.TERMS)
    spread = np.abs(m - m[:, :1, :1]).max()
    assert (spread > 0.1) if grows else (spread < 1e-5)
