"""Differentiable LLG trajectories (inverse problems, Sec. 4 of the paper).

LLGTrajectory.apply(theta, m0, mesh, dt, nsteps, ckpt_every, sample_every,
terms) runs nsteps fixed RK4 steps through the C ABI with the per-cell
applied-field map theta (float32 device tensor, shape (3, N3, N2, N1)) and
returns the states after every `sample_every`-th step, shape
(nsteps // sample_every, 3, N3+1, N2+1, N1+1).  Any torch loss of those
samples can be back-propagated: the backward pass walks the checkpoints
(every `ckpt_every` steps) from last to first and calls nm_adjoint_step,
which recomputes the segment and runs the exact discrete adjoint on the GPU.
Gradients flow to theta and m0.  This module only marshals arguments.
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
        theta = theta.detach().contiguous()
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
        ctx.save_for_backward(*ckpts)
        ctx.theta_shape = theta.shape
        return torch.stack(samples)

    @staticmethod
    def backward(ctx, grad_samples):
        dt, nsteps, ckpt_every, sample_every, terms, t0 = ctx.args
        ckpts = ctx.saved_tensors
        mesh = ctx.mesh
        g = grad_samples.contiguous()
        lam = torch.zeros_like(ckpts[0])
        gth = torch.zeros(ctx.theta_shape, dtype=torch.float32, device=lam.device)
        for si in range(len(ckpts) - 1, -1, -1):
            k0 = si * ckpt_every
            nseg = min(ckpt_every, nsteps - k0)
            dl = g[k0 // sample_every:(k0 + nseg) // sample_every]
            B.nm_adjoint_step(mesh, ckpts[si], t0 + k0 * dt, dt, nseg, terms, lam,
                              dl_dm=dl, dl_every=sample_every, grad_hcell=gth,
                              work=_workspace(mesh, nseg, lam.device))
        return gth, lam, None, None, None, None, None, None, None
