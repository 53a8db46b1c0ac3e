"""Domain-wall depinning at a two-phase boundary on the GPU (the second
validation of Sec. "Validation", Tab. sp_dw).

A wall sits in the soft phase of a chain of cells (soft phase, then hard
phase; `synth.two_phase_chain`).  A uniform field -H z pushes it against the
phase boundary; the depinning field is the smallest H at which it passes
into the hard phase.  It is found by bisection over H: each trial integrates
the LLG equation (DP45, alpha = 1, exchange + anisotropy + Zeeman) for a
fixed time from the last state that stayed pinned (quasi-static warm
starts), and the wall has depinned when the mean m_z of the hard phase's
nodes has turned negative.  A trial just above the threshold needs a long
time to pass the bottleneck, so the estimate is biased upwards by the field
excess whose passage time equals the trial time.

Every step runs in the library's kernels through the C ABI; the bisections
of several chains run in threads, each on its own mesh and stream.
"""
import math
from concurrent.futures import ThreadPoolExecutor

from . import binding as B

MU0 = 4e-7 * math.pi
TERMS = B.NM_T_EXCHANGE | B.NM_T_ANIS | B.NM_T_ZEEMAN


class _Chain:
    def __init__(self, p, device):
        import torch

        self.torch = torch
        self.stream = torch.cuda.Stream(device=device)
        self.mesh = B.mesh_from_problem(p, device=device, stream=self.stream, tensor=False)
        self.n_soft = int(p["n_soft"])
        self.cells = tuple(reversed(p["n"]))
        with torch.cuda.stream(self.stream):
            self.m = torch.as_tensor(p["m0"], device=device).contiguous()
            self.field = torch.zeros((3,) + self.cells, device=device)

    def trial(self, m_start, b, t_relax, dt0, rtol, atol):
        """Relax from m_start under mu0 H = b (T) along -z for t_relax; the
        final state and whether the wall has left the interface."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.field[2].fill_(-b / MU0)
            B.nm_mesh_set_field(self.mesh, self.field)
            m = m_start.clone()
            clk = B.nm_clock(0.0, dt0, 0, 0, 0, 0.0)
            B.nm_llg_step(self.mesh, m, clk, B.NM_DP45, TERMS, t_end=t_relax, rtol=rtol, atol=atol)
            mz_hard = float(m[2][..., self.n_soft:].mean())
        return m, mz_hard < 0.0, clk

    def close(self):
        B.nm_mesh_destroy(self.mesh)


def _bisect(ch, b_lo, b_hi, rel_tol, log, **kw):
    m, gone, clk = ch.trial(ch.m, b_lo, **kw)
    if log is not None:
        log.append((b_lo, gone, clk.accepted))
    if gone:
        raise RuntimeError("wall not pinned at the lower end of the bracket")
    _, gone, clk = ch.trial(m, b_hi, **kw)
    if log is not None:
        log.append((b_hi, gone, clk.accepted))
    if not gone:
        raise RuntimeError("wall still pinned at the upper end of the bracket")
    lo, hi = b_lo, b_hi
    while hi - lo > rel_tol * hi:
        mid = 0.5 * (lo + hi)
        t, gone, clk = ch.trial(m, mid, **kw)
        if log is not None:
            log.append((mid, gone, clk.accepted))
        if gone:
            hi = mid
        else:
            lo, m = mid, t
    return lo, hi


def depinning_fields(problems, brackets, rel_tol=2e-3, t_relax=5e-9, dt0=1e-13, rtol=1e-5, atol=1e-5,
                     device="cuda:0", logs=None):
    """Bisection for the depinning field of each two-phase chain problem (a
    `synth.two_phase_chain` dict), all chains at once: one thread, mesh and
    stream each.  brackets[i] = (b_lo, b_hi) in T, pinned at b_lo and
    depinned at b_hi (both checked).  Returns (lo, hi) per chain with
    hi - lo <= rel_tol hi.  logs, if given, is a list of lists receiving
    (b, depinned, accepted steps) per trial."""
    chains = []
    try:
        for p in problems:   # set-up one mesh at a time
            chains.append(_Chain(p, device))
        kw = dict(t_relax=t_relax, dt0=dt0, rtol=rtol, atol=atol)

        def run(i):
            return _bisect(chains[i], *brackets[i], rel_tol, None if logs is None else logs[i], **kw)

        with ThreadPoolExecutor(max_workers=len(chains)) as ex:
            return list(ex.map(run, range(len(chains))))
    finally:
        for ch in chains:
            ch.close()


def depinning_field(p, b_lo, b_hi, **kw):
    """depinning_fields for one chain."""
    logs = kw.pop("log", None)
    return depinning_fields([p], [(b_lo, b_hi)], logs=None if logs is None else [logs], **kw)[0]
