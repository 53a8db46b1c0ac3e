"""Glue between the seeded problems and the oracle, and closed forms the tests share (tests only)."""
import numpy as np

import oracle


def to_oracle(p):
    """Mesh and float64 Material from a problem dict of float32 arrays."""
    mesh = oracle.Mesh(p["n"], p["h"], basis=p.get("basis", "3d"))
    f = lambda a: None if a is None else np.asarray(a, dtype=np.float64)
    mat = oracle.Material(
        Ms=f(p["Ms"]), A=f(p["A"]), alpha=f(p["alpha"]), gamma=p["gamma"],
        Ku=f(p["Ku"]), easy=f(p["easy"]), h_cell=f(p["h_cell"]),
        h_uniform=f(p["h_uniform"]), drive_mask=f(p["drive_mask"]),
        drive_amp=f(p["drive_amp"]), drive_freq=p["drive_freq"],
        drive_phase=p["drive_phase"], D=f(p.get("D")), dmi_type=p.get("dmi_type", "interfacial"),
        Kc=f(p.get("Kc")),
        cubic=None if p.get("cubic") is None else f(p["cubic"]).reshape((2, 3) + tuple(p["cubic"].shape[1:])))
    return mesh, mat, np.asarray(p["m0"], dtype=np.float64)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def aharoni_factor(a, b, c):
    """Demagnetising factor along c of a uniformly magnetised rectangular
    prism of edges 2a x 2b x 2c (A. Aharoni, J. Appl. Phys. 83, 3432 (1998),
    the closed form of the body-averaged field)."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    t = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((ab + a) / (ab - a)) + a / (2 * c) * np.log((ab + b) / (ab - b))
         + c / (2 * a) * np.log((bc - b) / (bc + b)) + c / (2 * b) * np.log((ac - a) / (ac + a))
         + 2 * np.arctan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return t / np.pi



def gpu_replay_steps(B, mesh, m, steps, terms, rtol=1e-5, atol=1e-5):
    """Make the GPU take a given list of accepted DP45 steps (t, dt) (the
    oracle's own): one call per step, starting at t with the proposal dt and
    ending at t + dt.  Returns the clock of the last call; every attempt must
    have been accepted."""
    rej = 0
    clk = None
    for t, dt in steps:
        clk = B.nm_clock(t, dt, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, terms, t_end=t + dt, rtol=rtol, atol=atol, max_steps=1)
        rej += clk.rejected
        assert clk.accepted == 1, (t, dt, clk.accepted)
    assert rej == 0, "the GPU rejected %d of the oracle's accepted steps" % rej
    return clk
