"""The device-side DP45 controller's stopping rules and failure reports,
through the C ABI: a relaxation stopped by the torque criterion (the reported
torque is the state's, and below the limit), a step size falling below
dt_min (NM_ESTEPSIZE, m at the last accepted state), and a non-finite state
(NM_ENONFINITE, m untouched).  Every case ends through the controller's own
flags, so every kernel exits normally."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def _problem():
    return synth.block(n=(32, 32, 8))     # random start, alpha = 1


def _max_torque(mesh, m):
    f = torch.empty_like(m)
    B.nm_llg_rhs(mesh, m, f, B.NM_T_ALL, 0.0)
    return float(torch.linalg.vector_norm(f, dim=0).max())


def test_torque_stop_ends_the_relaxation_early():
    p = _problem()
    mesh = B.mesh_from_problem(p)
    try:
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        start = _max_torque(mesh, m)
        limit = 1e-2 * start
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=20e-9, stop_torque=limit,
                      max_steps=20000)
        end = _max_torque(mesh, m)
    finally:
        B.nm_mesh_destroy(mesh)
    assert 0 < clk.t < 20e-9 and clk.accepted < 20000
    assert clk.max_torque < limit
    assert abs(end - clk.max_torque) <= 1e-3 * clk.max_torque


def test_step_size_below_dt_min_is_reported_with_the_last_accepted_state():
    p = _problem()
    mesh = B.mesh_from_problem(p)
    try:
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        with pytest.raises(B.NMError) as err:
            # the stability limit of the exchange modes of 2 nm cells is a
            # few 1e-13 s, and a step grows at most 5-fold: the first
            # proposal falls below 1e-11 s
            B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=20e-9, dt_min=1e-11)
        # the same run stopped after its accepted steps (none or the first)
        ref = torch.as_tensor(p["m0"], device="cuda").contiguous()
        c1 = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        if clk.accepted:
            B.nm_llg_step(mesh, ref, c1, B.NM_DP45, B.NM_T_ALL, t_end=20e-9, max_steps=clk.accepted)
        torch.cuda.synchronize()
        same = torch.equal(m, ref)
    finally:
        B.nm_mesh_destroy(mesh)
    assert err.value.status == B.NM_ESTEPSIZE
    assert clk.accepted <= 1 and clk.t == c1.t
    assert same


def test_non_finite_state_is_reported_and_m_is_left_alone():
    p = _problem()
    p["m0"] = p["m0"].copy()
    p["m0"][:, 3, 10, 7] = np.nan
    mesh = B.mesh_from_problem(p)
    try:
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        before = m.clone()
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        with pytest.raises(B.NMError) as err:
            B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=1e-12)
        torch.cuda.synchronize()
        same = torch.equal(torch.nan_to_num(m, nan=7.0), torch.nan_to_num(before, nan=7.0))
    finally:
        B.nm_mesh_destroy(mesh)
    assert err.value.status == B.NM_ENONFINITE
    assert clk.accepted == 0 and same
