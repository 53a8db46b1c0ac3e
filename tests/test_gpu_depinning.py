"""Two-phase depinning on the GPU (the second validation of Sec.
"Validation", Tab. sp_dw, on chains of our own parameters): the field of a
chain with jumps in A, K and Ms against the float64 oracle, and the
depinning fields found by LLG relaxations on the GPU against the oracle's
discrete thresholds (energy minimisation of the same discretisation,
`tests/golden/depinning_fields.txt`).  The GPU bisection stops at a relative
bracket of 2e-3 and its trial time biases it upwards; 1% covers both."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.field import ANISOTROPY, EXCHANGE, ZEEMAN
from helpers import rel_l2, to_oracle
from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import depinning, synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depinning_fields.txt")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def _golden():
    rows = [ln.split() for ln in open(GOLDEN) if not ln.startswith("#")]
    return {(r[0], float(r[1])): tuple(map(float, r[2:])) for r in rows}


@pytest.mark.parametrize("case", ["A/K/Ms", "A/Ms", "K"])
def test_chain_field_matches_oracle(case):
    """The field across the phase boundary (the wall straddling it) with the
    depinning field's Zeeman term."""
    p = synth.two_phase_chain(case, hx=1e-9, soft_len=20e-9, hard_len=10e-9)
    p["h_uniform"] = np.array([0.0, 0.0, -0.5 / depinning.MU0], dtype=np.float32)
    terms = EXCHANGE | ANISOTROPY | ZEEMAN
    mesh = B.mesh_from_problem(p, tensor=False)
    try:
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        h = torch.empty_like(m)
        B.nm_heff(mesh, m, h, depinning.TERMS, 0.0)
        torch.cuda.synchronize()
        g = h.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    om, omat, m0 = to_oracle(p)
    assert rel_l2(g, oracle.heff(om, omat, m0, terms)) <= 1e-5


@pytest.mark.parametrize("hx", [1e-9, 0.5e-9])
def test_depinning_fields_match_oracle(hx):
    gold = _golden()
    cases = synth.DEPIN_CASES if hx == 1e-9 else ("A/K/Ms", "K")
    problems = [synth.two_phase_chain(c, hx=hx) for c in cases]
    brackets = [(0.5 * gold[(c, hx)][0], 1.5 * gold[(c, hx)][0]) for c in cases]
    got = depinning.depinning_fields(problems, brackets, rel_tol=2e-3, t_relax=5e-9)
    for c, (lo, hi) in zip(cases, got):
        bc, olo, ohi = gold[(c, hx)]
        b, ob = 0.5 * (lo + hi), 0.5 * (olo + ohi)
        print("%-7s hx %.1e  closed %.4f  oracle %.4f  gpu %.4f" % (c, hx, bc, ob, b))
        assert abs(b - ob) <= 1e-2 * ob, c
