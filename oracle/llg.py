"""LLG right-hand side and time integrators (oracle; float64).

* Eq. (llg): dm/dt = -gamma/(1+alpha^2) m x H - alpha gamma/(1+alpha^2) m x (m x H),
  evaluated node by node with the nodal damping (Ms-weighted cell mean).
* Sec. 5.3: classical RK4 with a fixed step and the adaptive Dormand-Prince
  5(4) pair (first-same-as-last) with an RMS error norm.

Controller (the paper names the method only): accept when the scaled RMS
error is <= 1; the next step is dt * clip(0.9 err^(-1/5), 0.2, 5), without
growth right after a rejection; the last step is shortened to land on t_end,
and a step that covers the remaining span to within a relative 1e-9 ends
the integration at t_end exactly (rounding in the sum of the steps leaves no
sliver step); the floor dt_min applies to the proposals of an integration
that goes on.
"""
import numpy as np

from .field import ALL_TERMS, heff, lumped_mass, nodal_alpha


def llg_rhs(mesh, mat, m, t=0.0, terms=ALL_TERMS, alpha_n=None):
    """f_n = -g' m x H - alpha g' m x (m x H), g' = gamma / (1 + alpha_n^2)."""
    H = heff(mesh, mat, m, terms, t)
    if alpha_n is None:
        alpha_n = nodal_alpha(mesh, mat)
    gp = mat.gamma / (1.0 + alpha_n ** 2)
    mxh = np.cross(m, H, axis=0)
    mxmxh = np.cross(m, mxh, axis=0)
    return -gp * mxh - alpha_n * gp * mxmxh


def rk4_step(mesh, mat, m, t, dt, terms=ALL_TERMS):
    a = nodal_alpha(mesh, mat)
    k1 = llg_rhs(mesh, mat, m, t, terms, a)
    k2 = llg_rhs(mesh, mat, m + 0.5 * dt * k1, t + 0.5 * dt, terms, a)
    k3 = llg_rhs(mesh, mat, m + 0.5 * dt * k2, t + 0.5 * dt, terms, a)
    k4 = llg_rhs(mesh, mat, m + dt * k3, t + dt, terms, a)
    return m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4_solve(mesh, mat, m0, dt, nsteps, t0=0.0, terms=ALL_TERMS, every=0):
    """Fixed-step RK4; returns m(t0 + nsteps dt) and snapshots every `every` steps."""
    m = np.array(m0, dtype=np.float64)
    snaps = []
    for k in range(nsteps):
        m = rk4_step(mesh, mat, m, t0 + k * dt, dt, terms)
        if every and (k + 1) % every == 0:
            snaps.append(m.copy())
    return m, snaps


class DP45:
    """Dormand & Prince (1980) RK5(4)7FM coefficients."""
    c = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])
    a = [
        [],
        [1 / 5],
        [3 / 40, 9 / 40],
        [44 / 45, -56 / 15, 32 / 9],
        [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
        [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
        [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
    ]
    b = np.array([35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0])
    bstar = np.array([5179 / 57600, 0.0, 7571 / 16695, 393 / 640,
                      -92097 / 339200, 187 / 2100, 1 / 40])


def error_norm(err, y_old, y_new, atol, rtol, active=None):
    """RMS over active node components of err / (atol + rtol max(|y_old|, |y_new|))."""
    sc = atol + rtol * np.maximum(np.abs(y_old), np.abs(y_new))
    r = (err / sc) ** 2
    if active is not None:
        r = r[:, active]
    return float(np.sqrt(np.mean(r)))


def dp45_attempt(mesh, mat, m, t, dt, k1=None, terms=ALL_TERMS, alpha_n=None):
    """One Dormand-Prince attempt: returns (y_new, err_vec, k7)."""
    if alpha_n is None:
        alpha_n = nodal_alpha(mesh, mat)
    T = DP45
    ks = [llg_rhs(mesh, mat, m, t, terms, alpha_n) if k1 is None else k1]
    for s in range(1, 7):
        y = m + dt * sum(T.a[s][j] * ks[j] for j in range(s) if T.a[s][j] != 0.0)
        ks.append(llg_rhs(mesh, mat, y, t + T.c[s] * dt, terms, alpha_n))
    y_new = m + dt * sum(T.b[j] * ks[j] for j in range(7) if T.b[j] != 0.0)
    err = dt * sum((T.b[j] - T.bstar[j]) * ks[j] for j in range(7))
    return y_new, err, ks[6]


def dp45_solve(mesh, mat, m0, t0, t_end, dt0, rtol=1e-5, atol=1e-5,
               terms=ALL_TERMS, dt_min=1e-20, dt_max=np.inf, max_attempts=100000,
               max_accepted=None, return_dt=False):
    """Adaptive DP45 from t0 to t_end; returns (m, log) with log the list of
    (t, dt, accepted) for every attempt, and with return_dt also the step the
    controller proposes next (to continue the integration in a later call).
    max_accepted: stop after that many accepted steps."""
    m = np.array(m0, dtype=np.float64)
    t, dt = float(t0), float(dt0)
    a = nodal_alpha(mesh, mat)
    active = lumped_mass(mesh, mat) > 0
    k1 = None
    log = []
    rejected_last = False
    n_acc = 0
    for _ in range(max_attempts):
        if t >= t_end or (max_accepted is not None and n_acc >= max_accepted):
            break
        dt = min(dt, t_end - t, dt_max)
        last = dt >= (t_end - t) * (1.0 - 1e-9)
        y, err, k7 = dp45_attempt(mesh, mat, m, t, dt, k1, terms, a)
        if k1 is None:
            k1 = llg_rhs(mesh, mat, m, t, terms, a)
        e = error_norm(err, m, y, atol, rtol, active)
        if not np.isfinite(e):
            raise FloatingPointError("non-finite error norm")
        fac = 5.0 if e == 0.0 else min(5.0, max(0.2, 0.9 * e ** -0.2))
        if e <= 1.0:
            log.append((t, dt, True))
            t = t_end if last else t + dt
            m = y
            k1 = k7
            if rejected_last:
                fac = min(fac, 1.0)
            rejected_last = False
            n_acc += 1
        else:
            log.append((t, dt, False))
            rejected_last = True
        dt = dt * fac
        if dt < dt_min and t < t_end:
            raise FloatingPointError("step size below dt_min")
    if return_dt:
        return m, log, dt
    return m, log


def dp45_replay(mesh, mat, m0, steps, terms=ALL_TERMS):
    """Take the 5th-order DP45 update for a given list of accepted (t, dt)."""
    m = np.array(m0, dtype=np.float64)
    a = nodal_alpha(mesh, mat)
    for t, dt in steps:
        m, _, _ = dp45_attempt(mesh, mat, m, t, dt, None, terms, a)
    return m
