"""Differentiable LLG trajectories (inverse problems, Sec. 4 of the paper).

LLGTrajectory.apply(theta, m0, mesh, dt, nsteps, ckpt_every, sample_every,
terms) runs nsteps fixed RK4 steps through the C ABI with the per-cell
applied-field map theta (float32 device tensor, shape (3, N3, N2, N1)) and
returns the states after every `sample_every`-th step, shape
(nsteps // sample_every, 3, N3+1, N2+1, N1+1).  Any torch loss of those
samples can be back-propagated: the backward pass walks the checkpoints
(every `ckpt_every` steps) from last to first and calls nm_adjoint_step,
which recomputes the segment and runs the exact discrete adjoint on the GPU.
Gradients flow to theta and m0.

LLGTrajectoryContinuous.apply(theta, m0, mesh, dt, nsteps, sample_every,
terms) returns the same samples but keeps only the final state: its backward
pass integrates the continuous adjoint system of Sec. 4 backwards with
nm_adjoint_continuous, rebuilding the trajectory as it goes and adding each
sample's loss gradient to the co-state at its time (the multi-time objective
the paper describes).  Memory stays that of the forward pass; the gradient
differs from the discrete one by O(dt^4).  This module only marshals
arguments.
"""
import torch

from . import binding as B

# adjoint workspaces kept per (mesh, segment length, size): the library
# records one graph per segment shape and workspace, so reusing the buffer
# lets later backward passes replay it instead of recording again
_WORKSPACES = {}


def _workspace(mesh, nsteps, device):
    nbytes = B.nm_adjoint_workspace_bytes(mesh, nsteps)
    key = (mesh.value, nsteps, nbytes, str(device))
    w = _WORKSPACES.get(key)
    if w is None:
        w = torch.empty(nbytes // 4, dtype=torch.float32, device=device)
        _WORKSPACES[key] = w
    return w


def release_workspaces():
    """Drop the cached adjoint workspaces (e.g. after destroying meshes)."""
    _WORKSPACES.clear()


class LLGTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, m0, mesh, dt, nsteps, ckpt_every, sample_every, terms, t0=0.0):
        if nsteps < 1 or ckpt_every < 1 or sample_every < 1:
            raise ValueError("nsteps, ckpt_every and sample_every must be >= 1")
        if ckpt_every % sample_every or nsteps % sample_every:
            raise ValueError("ckpt_every and nsteps must be multiples of sample_every")
        theta = theta.detach().clone().contiguous()   # kept for the backward pass
        B.nm_mesh_set_field(mesh, theta)
        m = m0.detach().clone().contiguous()
        ckpts, samples = [], []
        clk = B.nm_clock(t0, dt, 0, 0, 0, 0.0)
        k = 0
        while k < nsteps:
            if k % ckpt_every == 0:
                ckpts.append(m.clone())
            nxt = k + sample_every
            B.nm_llg_step(mesh, m, clk, B.NM_RK4, terms, t_end=t0 + nxt * dt, max_steps=sample_every)
            samples.append(m.clone())
            k = nxt
        ctx.mesh = mesh
        ctx.args = (dt, nsteps, ckpt_every, sample_every, terms, t0)
        ctx.save_for_backward(theta, *ckpts)
        return torch.stack(samples)

    @staticmethod
    def backward(ctx, grad_samples):
        dt, nsteps, ckpt_every, sample_every, terms, t0 = ctx.args
        theta, *ckpts = ctx.saved_tensors
        mesh = ctx.mesh
        # the adjoint recomputes the forward segments from the mesh's field
        # map: restore this trajectory's one (another forward pass on the
        # same mesh may have replaced it since)
        B.nm_mesh_set_field(mesh, theta)
        g = grad_samples.contiguous()
        lam = torch.zeros_like(ckpts[0])
        gth = torch.zeros(theta.shape, dtype=torch.float32, device=lam.device)
        for si in range(len(ckpts) - 1, -1, -1):
            k0 = si * ckpt_every
            nseg = min(ckpt_every, nsteps - k0)
            dl = g[k0 // sample_every:(k0 + nseg) // sample_every]
            B.nm_adjoint_step(mesh, ckpts[si], t0 + k0 * dt, dt, nseg, terms, lam,
                              dl_dm=dl, dl_every=sample_every, grad_hcell=gth,
                              work=_workspace(mesh, nseg, lam.device))
        return gth, lam, None, None, None, None, None, None, None


class LLGTrajectoryContinuous(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, m0, mesh, dt, nsteps, sample_every, terms, t0=0.0):
        if nsteps < 1 or sample_every < 1 or nsteps % sample_every:
            raise ValueError("nsteps must be a positive multiple of sample_every >= 1")
        theta = theta.detach().clone().contiguous()   # kept for the backward pass
        B.nm_mesh_set_field(mesh, theta)
        m = m0.detach().clone().contiguous()
        samples = []
        clk = B.nm_clock(t0, dt, 0, 0, 0, 0.0)
        for k in range(sample_every, nsteps + 1, sample_every):
            B.nm_llg_step(mesh, m, clk, B.NM_RK4, terms, t_end=t0 + k * dt, max_steps=sample_every)
            samples.append(m.clone())
        ctx.mesh = mesh
        ctx.args = (dt, nsteps, sample_every, terms, t0)
        ctx.save_for_backward(theta, m)
        return torch.stack(samples)

    @staticmethod
    def backward(ctx, grad_samples):
        dt, nsteps, sample_every, terms, t0 = ctx.args
        theta, m_end = ctx.saved_tensors
        B.nm_mesh_set_field(ctx.mesh, theta)   # this trajectory's field map
        g = grad_samples.contiguous()
        m = m_end.clone()
        a = torch.zeros_like(m)
        gth = torch.zeros(theta.shape, dtype=torch.float32, device=m.device)
        for si in range(nsteps // sample_every - 1, -1, -1):
            a += g[si]
            B.nm_adjoint_continuous(ctx.mesh, m, t0 + (si + 1) * sample_every * dt, dt, sample_every, terms, a,
                                    grad_hcell=gth)
        return gth, a, None, None, None, None, None, None
