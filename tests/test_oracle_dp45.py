"""Pins of the oracle's adaptive Dormand-Prince error norm and step controller
(Sec. 5.3 names the method; the norm and the controller follow the reading
recorded with the oracle: RMS over the components of magnetic nodes of
e / (atol + rtol max(|y_old|, |y_new|)), accept when <= 1, next step
dt clip(0.9 err^(-1/5), 0.2, 5), no growth right after a rejection, the last
step shortened to land on t_end exactly).

The pins do not go through the oracle's stage arithmetic.  An undamped
macrospin in a static field along z is a linear system: the in-plane part
w = m_x + i m_y obeys dw/dt = i gamma H w (exchange vanishes for uniform m
and a cube's self field is parallel to m), and m_z stays constant.  One
attempt of an explicit Runge-Kutta method multiplies w by the method's
stability polynomial R(z), z = i gamma H dt, so the 5th-order update is
R5(z) w and the embedded error is (R5(z) - R4(z)) w, with R5 and R4 the
polynomials of the weights b and b* (the first-same-as-last stage
included).  The error norm of every attempt, and with it the whole
accept / reject sequence of the controller, then follows in closed form.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle.field import EXCHANGE, ZEEMAN
from oracle.llg import DP45

GAMMA = 2.211e5
H = 1e5                      # A/m along z
# exchange and Zeeman with A = 0: exactly linear (the demag self field of a
# cube is parallel to m only to the ~1e-12 accuracy of its tensor, and with
# A > 0 steps this long would be far outside the stability region of the
# exchange modes, which amplify rounding-level non-uniformity of the nodes)
TERMS = EXCHANGE | ZEEMAN
THETA0, PHI0 = np.pi / 3, 0.3

# Dormand & Prince (1980), RK5(4)7FM: the published coefficient table
A_DP = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
B5 = [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), F(0)]
B4 = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200), F(187, 2100), F(1, 40)]


def _poly(b):
    """Coefficients of R(z) = 1 + sum_k z^k b^T A^(k-1) 1 (exact fractions)."""
    A = [[F(0)] * 7 for _ in range(7)]
    for i, row in enumerate(A_DP):
        for j, v in enumerate(row):
            A[i][j] = v
    v = [F(1)] * 7
    out = [F(1)]
    for _ in range(7):
        out.append(sum(bi * vi for bi, vi in zip(b, v)))
        v = [sum(A[i][j] * v[j] for j in range(7)) for i in range(7)]
    return out


R5 = _poly(B5)
R4 = _poly(B4)


def _R(coef, z):
    return sum(float(c) * z ** k for k, c in enumerate(coef))


def test_oracle_tableau_is_the_published_one():
    for i, row in enumerate(A_DP):
        assert np.allclose(DP45.a[i], [float(v) for v in row], rtol=0, atol=1e-16)
    assert np.allclose(DP45.b, [float(v) for v in B5], rtol=0, atol=1e-16)
    assert np.allclose(DP45.bstar, [float(v) for v in B4], rtol=0, atol=1e-16)


def test_stability_polynomials():
    """R5 is the published 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/120 + z^6/600;
    the embedded weights agree with exp(z) to order 4 only."""
    assert R5 == [F(1), F(1), F(1, 2), F(1, 6), F(1, 24), F(1, 120), F(1, 600), F(0)]
    assert R4[:5] == [F(1), F(1), F(1, 2), F(1, 6), F(1, 24)]
    assert R4[5] != F(1, 120)


def _macrospin(vacuum=False):
    """One cubic cell (8 nodes) with uniform m in a field along z, alpha = 0, A = 0;
    with vacuum, the same cell between two empty cells (Ms = 0) whose outer
    nodes carry no mass."""
    n = (3, 1, 1) if vacuum else (1, 1, 1)
    mesh = oracle.Mesh(n, (3e-9, 3e-9, 3e-9))
    cs = mesh.cell_shape
    Ms = np.full(cs, 8e5)
    if vacuum:
        Ms[..., 0] = Ms[..., 2] = 0.0
    mat = oracle.Material(Ms=Ms, A=np.zeros(cs), alpha=np.zeros(cs), gamma=GAMMA,
                          h_uniform=np.array([0.0, 0.0, H]))
    m0 = np.array([np.sin(THETA0) * np.cos(PHI0), np.sin(THETA0) * np.sin(PHI0), np.cos(THETA0)])
    m = np.broadcast_to(m0.reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
    return mesh, mat, m


def _closed_norm(w, mz, dt, atol, rtol):
    """Error norm of one attempt from state (w, mz) with step dt, and R5 w."""
    z = 1j * GAMMA * H * dt
    wn = _R(R5, z) * w
    e = (_R(R5, z) - _R(R4, z)) * w
    sx = atol + rtol * max(abs(w.real), abs(wn.real))
    sy = atol + rtol * max(abs(w.imag), abs(wn.imag))
    # the z component has no error; RMS over the three components
    return np.sqrt(((e.real / sx) ** 2 + (e.imag / sy) ** 2 + 0.0) / 3.0), wn


@pytest.mark.parametrize("dt", [2e-12, 1e-11, 4e-11])
def test_attempt_is_the_stability_polynomial(dt):
    mesh, mat, m = _macrospin()
    y, err, k7 = oracle.dp45_attempt(mesh, mat, m, 0.0, dt, terms=TERMS)
    w = m[0] + 1j * m[1]
    z = 1j * GAMMA * H * dt
    assert np.abs((y[0] + 1j * y[1]) - _R(R5, z) * w).max() <= 1e-13
    assert np.abs(y[2] - m[2]).max() <= 1e-13
    assert np.abs((err[0] + 1j * err[1]) - (_R(R5, z) - _R(R4, z)) * w).max() <= 1e-15
    assert np.abs(err[2]).max() <= 1e-15
    # first same as last: k7 is the right-hand side at the new state
    assert np.abs(k7 - oracle.llg_rhs(mesh, mat, y, terms=TERMS)).max() <= 1e-9 * np.abs(k7).max()


@pytest.mark.parametrize("atol,rtol", [(1e-5, 1e-5), (1e-6, 1e-4), (1e-3, 0.0)])
@pytest.mark.parametrize("vacuum", [False, True])
def test_error_norm_closed_form(atol, rtol, vacuum):
    """RMS over the components of the magnetic nodes: nodes without mass
    (vacuum) neither add error nor count in the mean."""
    mesh, mat, m = _macrospin(vacuum)
    active = oracle.lumped_mass(mesh, mat) > 0
    assert active.sum() == 8
    dt = 1.5e-11
    y, err, _ = oracle.dp45_attempt(mesh, mat, m, 0.0, dt, terms=TERMS)
    got = oracle.error_norm(err, m, y, atol, rtol, active)
    w = complex(m[0, 0, 0, 0], m[1, 0, 0, 0])
    want, _ = _closed_norm(w, m[2, 0, 0, 0], dt, atol, rtol)
    assert abs(got - want) <= 1e-10 * want


def _controller_log(dt0, t_end, atol, rtol):
    """The reading's controller applied to the closed-form error of each
    attempt (written out independently of the oracle's solver)."""
    w = np.sin(THETA0) * np.exp(1j * PHI0)
    mz = np.cos(THETA0)
    t, dt, rejected_last = 0.0, dt0, False
    log, capped = [], 0
    while t < t_end:
        dt = min(dt, t_end - t)
        last = dt >= (t_end - t) * (1.0 - 1e-9)
        err, wn = _closed_norm(w, mz, dt, atol, rtol)
        grow = min(5.0, max(0.2, 0.9 * err ** (-1.0 / 5.0)))
        if err <= 1.0:
            log.append((t, dt, True))
            t, w = (t_end if last else t + dt), wn
            if rejected_last and grow > 1.0:
                capped += 1
                grow = 1.0
            rejected_last = False
        else:
            log.append((t, dt, False))
            rejected_last = True
        dt *= grow
    return log, w, capped


@pytest.mark.parametrize("vacuum", [False, True])
def test_controller_follows_the_closed_form_errors(vacuum):
    """A forced rejection (dt0 far too large), the no-growth rule right after
    it, the steady step and the shortened last step: the oracle's attempt
    log equals the rule applied to the closed-form errors."""
    atol = rtol = 1e-5
    # dt0 = 1e-10: the error (~1.5e3) is where the z^6, z^7 terms steepen
    # it, so the retry after the rejection lands below the steady step and
    # the no-growth rule binds
    dt0, t_end = 1e-10, 1e-9
    want, w_end, capped = _controller_log(dt0, t_end, atol, rtol)
    assert sum(1 for x in want if not x[2]) >= 1 and capped >= 1
    assert len(want) > 20
    mesh, mat, m = _macrospin(vacuum)
    mT, got = oracle.dp45_solve(mesh, mat, m, 0.0, t_end, dt0, rtol=rtol, atol=atol, terms=TERMS)
    assert len(got) == len(want)
    for (tg, dg, ag), (tw, dw, aw) in zip(got, want):
        assert ag == aw
        # the embedded error is a difference of nearly equal stage sums, so
        # the oracle's norm carries ~1e-10 relative rounding; a change of the
        # rule moves a step by a percent or more
        assert abs(tg - tw) <= 1e-9 * t_end and abs(dg - dw) <= 1e-9 * dw
    act = oracle.lumped_mass(mesh, mat) > 0
    assert np.abs(mT[0][act] + 1j * mT[1][act] - w_end).max() <= 1e-11


def test_controller_bounds_the_step_change():
    """A zero error grows the step by the cap of 5; a huge one shrinks it by
    the floor of 0.2 (a static field along m: no torque, no error)."""
    mesh, mat, m = _macrospin()
    m[...] = 0.0
    m[2] = 1.0
    _, log = oracle.dp45_solve(mesh, mat, m, 0.0, 1e-9, 1e-13, terms=TERMS)
    dts = [dt for _, dt, _ in log]
    assert all(ok for _, _, ok in log)
    assert abs(dts[1] / dts[0] - 5.0) <= 1e-12 and abs(dts[2] / dts[1] - 5.0) <= 1e-12
    mesh, mat, m = _macrospin()
    _, log = oracle.dp45_solve(mesh, mat, m, 0.0, 1e-9, 4e-10, max_accepted=1, terms=TERMS)
    assert not log[0][2] and abs(log[1][1] / log[0][1] - 0.2) <= 1e-12


def test_max_accepted_and_continuation():
    """Stopping after k accepted steps and continuing from the returned
    proposal reproduces one uninterrupted run's steps."""
    mesh, mat, m = _macrospin()
    _, full = oracle.dp45_solve(mesh, mat, m, 0.0, 4e-10, 5e-11, terms=TERMS)
    m1, a, dt = oracle.dp45_solve(mesh, mat, m, 0.0, 4e-10, 5e-11, max_accepted=3, return_dt=True,
                                     terms=TERMS)
    t1 = a[-1][0] + a[-1][1]
    _, b = oracle.dp45_solve(mesh, mat, m1, t1, 4e-10, dt, terms=TERMS)
    acc = [x for x in a if x[2]]
    assert len(acc) == 3
    # the continuation forgets a rejection just before the split only; here
    # the third accepted step is not preceded by one
    assert [x[1] for x in a + b] == pytest.approx([x[1] for x in full], rel=1e-12)


def test_last_step_lands_on_t_end_under_a_step_cap():
    """With a step cap that does not divide the span, the steps add up to
    t_end without a rounding sliver: the last one ends exactly there and no
    step-size floor is hit on the way out (a sliver step of ~1e-26 s would
    propose a step below dt_min)."""
    mesh, mat, m = _macrospin()
    span = 1e-9
    _, log = oracle.dp45_solve(mesh, mat, m, 0.0, span, 1e-13, dt_max=3e-13, dt_min=1e-20, terms=TERMS)
    acc = [(t, dt) for t, dt, ok in log if ok]
    assert all(dt > 1e-14 for _, dt in acc)
    assert acc[-1][0] + acc[-1][1] == pytest.approx(span, rel=1e-12)
    assert max(dt for _, dt in acc) <= 3e-13
    _, log2, dt_next = oracle.dp45_solve(mesh, mat, m, 0.0, span, 1e-13, dt_max=3e-13, terms=TERMS,
                                         return_dt=True)
    assert dt_next > 0 and log2 == log
