"""Discrete adjoint of the RK4-integrated LLG equation (oracle; float64).

The paper's inverse problems (Sec. 4, Eqs. adjoint_forward, adjoint_objective,
adjoint_system) need the gradient of an objective over a trajectory with
respect to design variables theta.  The oracle differentiates the discrete
map (discretise first, as the paper does for static problems): for every
RK4 step it runs the exact reverse recurrence of the four stages.

Ingredients, written out from the definitions:
  * VJP of the LLG right-hand side f(m, H) = -g' m x H - a g' m x (m x H)
    (g' = gamma / (1 + alpha^2), a = alpha) for a co-vector w:
        df/dm^T w = -g' H x w - a g' [ H (w.m) + (m.H) w - 2 m (w.H) ]
        u := df/dH^T w = g' m x w - a g' [ (m.w) m - |m|^2 w ]
  * the field H(m) = H_lin(m) + H_ext(theta, t) with H_lin = -M^-1 K m for
    the quadratic energies (exchange, anisotropy, demag; K symmetric), so
    dH/dm^T u = -K M^-1 u = M H_lin(M^-1 u): the backward field is the
    forward linear field of a rescaled vector;
  * theta = per-cell applied field map: H_ext,n = sum_{c containing n}
    (mu0 Ms_c V/8 / M_n) theta_c, so dL/dtheta_c = sum_{n in c} mu0 Ms_c V/8
    (M^-1 u)_n.
"""
import numpy as np

from .field import CUBIC, ZEEMAN, heff, lumped_mass, nodal_alpha
from .mesh import MU0


def llg_vjp(m, H, w, alpha_n, gp):
    """(df/dm^T w, df/dH^T w) of the LLG right-hand side, node by node."""
    a = gp
    b = alpha_n * gp
    wm = np.sum(w * m, axis=0)
    mH = np.sum(m * H, axis=0)
    wH = np.sum(w * H, axis=0)
    mm = np.sum(m * m, axis=0)
    dm = -a * np.cross(H, w, axis=0) - b * (H * wm + mH * w - 2.0 * m * wH)
    u = a * np.cross(m, w, axis=0) - b * (wm * m - mm * w)
    return dm, u


def cell_gather(mesh, mat, v):
    """dL/dtheta_c = mu0 Ms_c V/8 sum_{n in c} v_n for the nodal v = M^-1 u."""
    acc = np.zeros((3,) + mesh.cell_shape)
    for a in mesh.corners:
        acc += mesh.corner(v, a)
    return MU0 * mat.Ms * mesh.V / len(mesh.corners) * acc


def rhs_vjp(mesh, mat, y, t, w, terms, alpha_n=None):
    """(df/dm^T w, dL/dtheta contribution) of f(y, t) for the co-vector w."""
    if terms & CUBIC and mat.Kc is not None:
        # the backward field reuses the forward one, which holds for the
        # quadratic energies only; the quartic cubic term is not covered
        raise NotImplementedError("the adjoint covers the quadratic energy terms")
    if alpha_n is None:
        alpha_n = nodal_alpha(mesh, mat)
    gp = mat.gamma / (1.0 + alpha_n ** 2)
    H = heff(mesh, mat, y, terms, t)
    dm, u = llg_vjp(y, H, w, alpha_n, gp)
    M = lumped_mass(mesh, mat)
    v = np.where(M > 0, u / np.where(M > 0, M, 1.0), 0.0)
    lin = terms & ~ZEEMAN
    if lin:
        dm = dm + M * heff(mesh, mat, v, lin, t)
    dth = cell_gather(mesh, mat, v) if terms & ZEEMAN else np.zeros((3,) + mesh.cell_shape)
    return dm, dth


def rk4_step_adjoint(mesh, mat, m, t, dt, lam, terms, alpha_n=None):
    """Given lam = dL/dm_{k+1}, return (dL/dm_k through this step, dL/dtheta).

    Forward: y1 = m, k_s = f(y_s, t_s), y2 = m + dt/2 k1, y3 = m + dt/2 k2,
    y4 = m + dt k3, m' = m + dt/6 (k1 + 2 k2 + 2 k3 + k4).  Reverse, with
    w_s the co-vector of k_s:
      w4 = dt/6 lam, w3 = dt/3 lam + dt J4^T w4, w2 = dt/3 lam + dt/2 J3^T w3,
      w1 = dt/6 lam + dt/2 J2^T w2, lam_k = lam + sum_s J_s^T w_s.
    """
    from .llg import llg_rhs
    if alpha_n is None:
        alpha_n = nodal_alpha(mesh, mat)
    y1 = m
    k1 = llg_rhs(mesh, mat, y1, t, terms, alpha_n)
    y2 = m + 0.5 * dt * k1
    k2 = llg_rhs(mesh, mat, y2, t + 0.5 * dt, terms, alpha_n)
    y3 = m + 0.5 * dt * k2
    k3 = llg_rhs(mesh, mat, y3, t + 0.5 * dt, terms, alpha_n)
    y4 = m + dt * k3
    w4 = dt / 6.0 * lam
    g4, th4 = rhs_vjp(mesh, mat, y4, t + dt, w4, terms, alpha_n)
    w3 = dt / 3.0 * lam + dt * g4
    g3, th3 = rhs_vjp(mesh, mat, y3, t + 0.5 * dt, w3, terms, alpha_n)
    w2 = dt / 3.0 * lam + 0.5 * dt * g3
    g2, th2 = rhs_vjp(mesh, mat, y2, t + 0.5 * dt, w2, terms, alpha_n)
    w1 = dt / 6.0 * lam + 0.5 * dt * g2
    g1, th1 = rhs_vjp(mesh, mat, y1, t, w1, terms, alpha_n)
    return lam + g1 + g2 + g3 + g4, th1 + th2 + th3 + th4


def rk4_gradient(mesh, mat, m0, dt, nsteps, dloss, terms, t0=0.0, lam_end=None):
    """Gradient of L = sum_{k=1..nsteps} l_k(m_k) by the discrete adjoint.

    dloss(k, m_k) returns dl_k/dm_k (k = 1..nsteps).  Returns
    (dL/dm_0, dL/dtheta, m_nsteps).  All states are stored (the oracle is not
    memory-limited)."""
    from .llg import rk4_step
    a = nodal_alpha(mesh, mat)
    states = [np.array(m0, dtype=np.float64)]
    for k in range(nsteps):
        states.append(rk4_step(mesh, mat, states[-1], t0 + k * dt, dt, terms))
    lam = np.zeros_like(states[0]) if lam_end is None else np.array(lam_end, dtype=np.float64)
    dth = np.zeros((3,) + mesh.cell_shape)
    for k in range(nsteps, 0, -1):
        lam = lam + dloss(k, states[k])
        lam, th = rk4_step_adjoint(mesh, mat, states[k - 1], t0 + (k - 1) * dt, dt, lam, terms, a)
        dth += th
    return lam, dth, states[-1]


def region_mz2_loss(mesh, region, nsteps):
    """L = -(1/nsteps) sum_k mean over region nodes of m_z(t_k)^2 and its
    per-step gradient; region is a boolean nodal mask (N3+1, N2+1, N1+1)."""
    cnt = float(region.sum())

    def loss(m):
        return -float(np.sum(np.where(region, m[2] ** 2, 0.0))) / cnt / nsteps

    def dloss(k, m):
        g = np.zeros_like(m)
        g[2] = np.where(region, -2.0 * m[2] / cnt / nsteps, 0.0)
        return g

    return loss, dloss


def continuous_adjoint(mesh, mat, m_end, t_end, dt, nsteps, a_end, terms, alpha_n=None):
    """The adjoint system of Sec. 4 (Eq. adjoint_system), integrated backwards.

    From t_end down to t_end - nsteps dt with classical RK4 steps of -dt on the
    joint state (m, a, u):
        dm/dt = f(t, m),   da/dt = -(df/dm)^T a,   du/dt = -(df/dtheta)^T a,
    with m(t_end) = m_end, a(t_end) = a_end = dL/dm(t_end) and u(t_end) = 0.
    The trajectory m is rebuilt by integrating the LLG equation backwards, so
    no forward state is stored.  Returns (m, a, u) at the earlier time: u is
    the gradient of L with respect to the field map theta, a the one with
    respect to the initial state."""
    from .llg import llg_rhs
    if alpha_n is None:
        alpha_n = nodal_alpha(mesh, mat)

    def F(t, m, a):
        f = llg_rhs(mesh, mat, m, t, terms, alpha_n)
        ja, jth = rhs_vjp(mesh, mat, m, t, a, terms, alpha_n)
        return f, -ja, -jth

    h = -float(dt)
    m = np.array(m_end, dtype=np.float64)
    a = np.array(a_end, dtype=np.float64)
    u = np.zeros((3,) + mesh.cell_shape)
    t = float(t_end)
    for _ in range(nsteps):
        f1, g1, q1 = F(t, m, a)
        f2, g2, q2 = F(t + 0.5 * h, m + 0.5 * h * f1, a + 0.5 * h * g1)
        f3, g3, q3 = F(t + 0.5 * h, m + 0.5 * h * f2, a + 0.5 * h * g2)
        f4, g4, q4 = F(t + h, m + h * f3, a + h * g3)
        m = m + h / 6.0 * (f1 + 2.0 * f2 + 2.0 * f3 + f4)
        a = a + h / 6.0 * (g1 + 2.0 * g2 + 2.0 * g3 + g4)
        u = u + h / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4)
        t = t + h
    return m, a, u
