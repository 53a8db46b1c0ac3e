"""Glue between the seeded problems and the oracle (tests only)."""
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
        drive_phase=p["drive_phase"], D=f(p.get("D")))
    return mesh, mat, np.asarray(p["m0"], dtype=np.float64)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
