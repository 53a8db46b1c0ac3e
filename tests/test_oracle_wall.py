"""Pin of the oracle's local terms by a closed form: a Bloch wall in a
uniform chain (exchange + uniaxial anisotropy, no demag) has the energy
4 sqrt(A K) per unit area and the profile theta = 2 atan(exp(-x / delta)),
delta = sqrt(A / K), reached by the discrete minimum at second order in the
cell size."""
import numpy as np

import oracle
from oracle import depinning as dp
from oracle.field import ANISOTROPY, EXCHANGE

from helpers import to_oracle
from paper_2411_11725_amd import synth

A, K = 1e-11, 1e6


def _relaxed_wall(hx):
    p = synth.wall_chain(hx=hx, length=40e-9, A=A, K=K)
    mesh, mat, m0 = to_oracle(p)
    th = dp.relax(mesh, mat, dp.column_angles(m0), 0.0)
    e = oracle.energies(mesh, mat, dp._m_of(mesh, th), EXCHANGE | ANISOTROPY)
    # relative to the uniform state, whose anisotropy energy is -K V
    e_wall = (e["exchange"] + e["anisotropy"] + K * mesh.V * mesh.n_cells) / (2 * hx * hx)
    return th, e_wall, mesh


def test_wall_energy_converges_to_4_sqrt_AK_at_second_order():
    want = 4 * np.sqrt(A * K)
    errs = [(_relaxed_wall(hx)[1] - want) / want for hx in (1e-9, 0.5e-9)]
    assert 0 < errs[1] < errs[0] < 3e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_wall_profile_is_the_closed_form():
    hx = 0.25e-9
    th, _, mesh = _relaxed_wall(hx)
    x = np.arange(mesh.n[0] + 1) * hx - 0.5 * mesh.n[0] * hx   # the wall stays centred by symmetry
    want = 2 * np.arctan(np.exp(-x / np.sqrt(A / K)))
    # within three widths of the centre (the free ends, six widths out, bend
    # the finite chain's tails away from the infinite wall's)
    inner = np.abs(x) <= 3 * np.sqrt(A / K)
    assert np.abs(th - want)[inner].max() <= 5e-4
