"""A Bloch wall relaxed by the GPU's LLG integration (DP45, alpha = 1,
exchange + anisotropy) against the oracle's discrete energy minimum of the
same chain and the closed form 4 sqrt(A K) per unit area."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import depinning as dp
from oracle.field import ANISOTROPY, EXCHANGE
from helpers import to_oracle
from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import synth

pytestmark = pytest.mark.gpu

A, K = 1e-11, 1e6
TERMS = B.NM_T_EXCHANGE | B.NM_T_ANIS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


@pytest.mark.parametrize("hx", [1e-9, 0.5e-9])
def test_relaxed_wall_energy(hx):
    p = synth.wall_chain(hx=hx, length=40e-9, A=A, K=K)
    mesh = B.mesh_from_problem(p, tensor=False)
    try:
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, TERMS, t_end=0.5e-9, rtol=1e-6, atol=1e-6)
        e = B.nm_energy(mesh, m, TERMS, 0.0)
        f = torch.empty_like(m)
        B.nm_llg_rhs(mesh, m, f, TERMS, 0.0)
        torch.cuda.synchronize()
        torque = float(f.abs().max())
    finally:
        B.nm_mesh_destroy(mesh)
    om, omat, m0 = to_oracle(p)
    uniform = K * om.V * om.n_cells
    area = 2 * hx * hx
    th = dp.relax(om, omat, dp.column_angles(m0), 0.0)
    eo = oracle.energies(om, omat, dp._m_of(om, th), EXCHANGE | ANISOTROPY)
    e_oracle = (eo["exchange"] + eo["anisotropy"] + uniform) / area
    e_gpu = (e["exchange"] + e["anisotropy"] + uniform) / area
    print("hx %.1e  torque %.3e 1/s  wall energy gpu %.6e oracle %.6e closed %.6e J/m^2"
          % (hx, torque, e_gpu, e_oracle, 4 * np.sqrt(A * K)))
    assert torque < 1e8                       # four orders below the start
    assert abs(e_gpu - e_oracle) <= 1e-4 * e_oracle
    assert abs(e_gpu / (4 * np.sqrt(A * K)) - 1) <= 3e-3
