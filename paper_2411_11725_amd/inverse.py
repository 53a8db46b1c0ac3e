"""The field-direction inverse problem of the paper's inverse-problems
section: find the direction (theta, phi) of an applied field of fixed
magnitude that brings a single-domain particle from its initial state to a
target magnetisation m_target at time T.

    H_ext(theta, phi) = H (sin theta cos phi, sin theta sin phi, cos theta)
    L(theta, phi) = mean over the nodes and components of (m(T) - m_target)^2

The trajectory and its gradient run on the GPU (LLGTrajectory: fixed RK4
steps through the C ABI and the discrete adjoint); the field enters as a
uniform per-cell field map, so autograd carries the map's gradient to the
two angles.  Parameters the paper leaves open (particle size, material,
damping, optimiser) are chosen here and stated in field_direction_problem.
"""
import math

import numpy as np
import torch

from . import binding as B
from . import synth
from .adjoint import LLGTrajectory

MU0_SI = 4.0e-7 * math.pi


def field_direction_problem(n=(4, 4, 4), h=2e-9, Ms=8.0e5, A=1.3e-11, Ku=5.0e5, alpha=0.5):
    """A 8 nm cube (single domain) with uniaxial anisotropy along z, m0 along
    +z; the applied field magnitude is half the anisotropy field
    Hc = 2 Ku / (mu0 Ms)."""
    zero = np.zeros((3, n[2], n[1], n[0]))
    p = synth.make_problem(n, (h, h, h), Ms, A, alpha, m0=(0.0, 0.0, 1.0), Ku=Ku, easy=(0.0, 0.0, 1.0),
                           h_cell=zero)
    return p, 2.0 * Ku / (MU0_SI * Ms)


def field_map(angles, H, cell_shape):
    """Uniform per-cell field map (3, N3, N2, N1) of the direction angles."""
    th, ph = angles[0], angles[1]
    v = torch.stack([torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph), torch.cos(th)]) * H
    return v.reshape(3, 1, 1, 1).expand((3,) + tuple(cell_shape)).contiguous()


def loss_and_grad(mesh, p, angles, H, m_target, T, dt,
                  terms=B.NM_T_EXCHANGE | B.NM_T_ANIS | B.NM_T_ZEEMAN):
    """L(angles) and dL/dangles (GPU forward and discrete adjoint)."""
    nsteps = int(round(T / dt))
    a = angles.detach().clone().requires_grad_(True)
    theta = field_map(a, H, (p["n"][2], p["n"][1], p["n"][0]))
    m0 = torch.as_tensor(p["m0"], device=a.device).contiguous()
    traj = LLGTrajectory.apply(theta, m0, mesh, dt, nsteps, nsteps, nsteps, terms)
    L = ((traj[-1] - m_target.reshape(3, 1, 1, 1)) ** 2).mean()
    L.backward()
    return float(L.detach()), a.grad.detach().clone()


def optimize_field_direction(T=0.05e-9, dt=5e-14, iters=50, lr=0.1, target=(0.5 ** 0.5, 0.0, 0.5 ** 0.5),
                             start=(math.pi / 2, math.pi / 2), device="cuda", tol=1e-6):
    """Gradient descent (Adam) on the two field angles from `start`; returns
    the angle and loss history (one entry per gradient evaluation)."""
    p, Hc = field_direction_problem()
    H = 0.5 * Hc
    mesh = B.mesh_from_problem(p, device=device, tensor=False)
    try:
        angles = torch.tensor(start, dtype=torch.float32, device=device)
        m_target = torch.tensor(target, dtype=torch.float32, device=device)
        opt_angles = angles.clone().requires_grad_(True)
        opt = torch.optim.Adam([opt_angles], lr=lr)
        hist = []
        for _ in range(iters):
            L, g = loss_and_grad(mesh, p, opt_angles.detach(), H, m_target, T, dt)
            a = opt_angles.detach()
            hist.append((L, a[0].item(), a[1].item()))
            if L < tol:
                break
            opt.zero_grad()
            opt_angles.grad = g
            opt.step()
        return hist
    finally:
        B.nm_mesh_destroy(mesh)
