"""Pins of the oracle on meshes with vacuum cells (Ms = 0): nodes of zero
lumped mass have H = 0 and dm/dt = 0, and a magnet embedded in vacuum has
the field, right-hand side and energies it has alone (the demag convolution
is linear, so the larger padded grid changes nothing)."""
import numpy as np

import oracle
from oracle.field import ALL_TERMS

from helpers import to_oracle
from paper_2411_11725_amd import synth

CORE = ((6, 5, 3), (2e-9, 2.5e-9, 3e-9))
BIG, OFF = (11, 9, 6), (3, 2, 1)


def _pair():
    p = synth.small_random(*CORE, seed=3, dmi=True)
    q = synth.embed_in_vacuum(p, BIG, OFF)
    return p, q


def _core_nodes(a):
    (n1, n2, n3), (o1, o2, o3) = CORE[0], OFF
    return a[..., o3:o3 + n3 + 1, o2:o2 + n2 + 1, o1:o1 + n1 + 1]


def test_embedding_in_vacuum_changes_nothing():
    p, q = _pair()
    mp, matp, m0p = to_oracle(p)
    mq, matq, m0q = to_oracle(q)
    hp = oracle.heff(mp, matp, m0p, ALL_TERMS)
    hq = oracle.heff(mq, matq, m0q, ALL_TERMS)
    assert np.abs(_core_nodes(hq) - hp).max() <= 1e-10 * np.abs(hp).max()
    fp = oracle.llg_rhs(mp, matp, m0p)
    fq = oracle.llg_rhs(mq, matq, m0q)
    assert np.abs(_core_nodes(fq) - fp).max() <= 1e-10 * np.abs(fp).max()
    ep, eq = oracle.energies(mp, matp, m0p), oracle.energies(mq, matq, m0q)
    for k in ep:
        assert abs(ep[k] - eq[k]) <= 1e-10 * max(abs(ep[k]), 1e-30), k


def test_vacuum_nodes_have_no_field_and_do_not_move():
    _, q = _pair()
    mq, matq, m0q = to_oracle(q)
    M = oracle.lumped_mass(mq, matq)
    vac = M == 0
    assert vac.sum() == np.prod(mq.node_shape) - np.prod(np.array(CORE[0]) + 1)
    assert not np.any(oracle.heff(mq, matq, m0q)[:, vac])
    assert not np.any(oracle.llg_rhs(mq, matq, m0q)[:, vac])
    m1 = oracle.rk4_step(mq, matq, m0q, 0.0, 1e-14)
    assert np.array_equal(m1[:, vac], m0q[:, vac])
