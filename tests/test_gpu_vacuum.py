"""Vacuum cells (Ms = 0) on the GPU, through the C ABI: a magnet embedded in
vacuum against the float64 oracle (field, right-hand side, energies, RK4,
and DP45 replay), vacuum nodes held at H = 0 and m unchanged, the embedded
magnet against the same magnet alone on the GPU (the same adaptive steps),
a porous mesh of random holes, and a mesh without magnetic cells refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.field import ALL_TERMS
from helpers import gpu_replay_steps, rel_l2, to_oracle
from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import synth

pytestmark = pytest.mark.gpu

CORE = ((6, 5, 3), (2e-9, 2.5e-9, 3e-9))
BIG, OFF = (11, 9, 6), (3, 2, 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _pair():
    p = synth.small_random(*CORE, seed=3, dmi=True)
    return p, synth.embed_in_vacuum(p, BIG, OFF)


def _core_nodes(a):
    (n1, n2, n3), (o1, o2, o3) = CORE[0], OFF
    return a[..., o3:o3 + n3 + 1, o2:o2 + n2 + 1, o1:o1 + n1 + 1]


def _eval(p, kind):
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        out = torch.empty_like(m)
        if kind == "heff":
            B.nm_heff(mesh, m, out, B.NM_T_ALL, 0.0)
        else:
            B.nm_llg_rhs(mesh, m, out, B.NM_T_ALL, 0.0)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)


def test_embedded_field_matches_oracle_and_the_magnet_alone():
    p, q = _pair()
    om, omat, m0 = to_oracle(q)
    vac = oracle.lumped_mass(om, omat) == 0
    for kind, ref in (("heff", oracle.heff(om, omat, m0)), ("rhs", oracle.llg_rhs(om, omat, m0))):
        g = _eval(q, kind)
        assert rel_l2(g, ref) <= 1e-5
        assert not np.any(g[:, vac])
        assert rel_l2(_core_nodes(g), _eval(p, kind)) <= 1e-5


def test_embedded_energies_match_oracle():
    _, q = _pair()
    om, omat, m0 = to_oracle(q)
    mesh = B.mesh_from_problem(q)
    try:
        e = B.nm_energy(mesh, _dev(q["m0"]), B.NM_T_ALL, 0.0)
    finally:
        B.nm_mesh_destroy(mesh)
    want = oracle.energies(om, omat, m0)
    scale = max(abs(want[k]) for k in ("exchange", "demag", "anisotropy", "zeeman", "dmi"))
    for k in ("exchange", "demag", "anisotropy", "zeeman", "dmi", "total"):
        assert abs(e[k] - want[k]) <= 1e-5 * scale, k


def test_embedded_rk4_matches_oracle_and_leaves_vacuum_untouched():
    _, q = _pair()
    om, omat, m0 = to_oracle(q)
    vac = oracle.lumped_mass(om, omat) == 0
    dt, ns = 2e-14, 20
    mesh = B.mesh_from_problem(q)
    try:
        m = _dev(q["m0"])
        clk = B.nm_clock(0.0, dt, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_RK4, B.NM_T_ALL, t_end=ns * dt)
        g = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    want = m0
    for k in range(ns):
        want = oracle.rk4_step(om, omat, want, k * dt, dt)
    assert np.abs(g - want).max() <= 1e-5
    assert np.array_equal(g[:, vac], np.asarray(q["m0"], dtype=np.float64)[:, vac])


def _dp45(p, max_steps):
    mesh = B.mesh_from_problem(p)
    log = torch.zeros(3 * 64, dtype=torch.float64, device="cuda")
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=1e-9, rtol=1e-5, atol=1e-5,
                      log=log, max_steps=max_steps)
        g = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    L = log.cpu().numpy().reshape(-1, 3)[: clk.accepted + clk.rejected]
    return g, [(t, dt) for t, dt, ok in L if ok > 0.5]


def test_dp45_error_norm_runs_over_magnetic_nodes_only():
    """The embedded magnet takes the steps the magnet alone takes: the error
    norm is the RMS over the same active nodes (counting the vacuum nodes
    would scale it by sqrt(168/720) and every step by ~16%).  The error
    estimate is a cancelling combination of the stage derivatives, which
    amplifies the rounding differences of the two meshes' FFTs to ~1e-4 in
    the step sizes.  The oracle's own run of the embedded magnet takes the
    same steps, and the GPU replaying the oracle's steps matches it node by
    node."""
    p, q = _pair()
    gp, sp = _dp45(p, 5)
    gq, sq = _dp45(q, 5)
    assert len(sp) == len(sq) == 5
    assert np.allclose(np.array(sq), np.array(sp), rtol=1e-3, atol=0)
    assert np.abs(_core_nodes(gq) - gp).max() <= 1e-4   # the same states at ~1e-4 different times
    om, omat, m0 = to_oracle(q)
    want, olog = oracle.dp45_solve(om, omat, m0, 0.0, 1e-9, 1e-14, rtol=1e-5, atol=1e-5, max_accepted=5)
    so = [(t, dt) for t, dt, ok in olog if ok]
    assert np.allclose(np.array(sq), np.array(so), rtol=1e-3, atol=0)
    mesh = B.mesh_from_problem(q)
    try:
        m = _dev(q["m0"])
        gpu_replay_steps(B, mesh, m, so, B.NM_T_ALL)
        gr = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    assert np.abs(gr - want).max() <= 1e-6


def test_porous_mesh_matches_oracle():
    """A fifth of the cells empty at random (isolated vacuum nodes among them)."""
    p = synth.small_random((14, 9, 4), (2e-9, 2e-9, 3e-9), seed=31, ku_range=(-5e5, 5e5), dmi=True)
    holes = np.random.default_rng(32).random(p["Ms"].shape) < 0.2
    p["Ms"] = np.ascontiguousarray(np.where(holes, 0.0, p["Ms"]).astype(np.float32))
    om, omat, m0 = to_oracle(p)
    assert np.any(oracle.lumped_mass(om, omat) == 0)
    assert rel_l2(_eval(p, "heff"), oracle.heff(om, omat, m0)) <= 1e-5
    assert rel_l2(_eval(p, "rhs"), oracle.llg_rhs(om, omat, m0)) <= 1e-5


def test_mesh_without_magnetic_cells_is_refused():
    p = synth.small_random((5, 4, 2), (2e-9,) * 3, seed=33)
    p["Ms"] = np.zeros_like(p["Ms"])
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        h = torch.empty_like(m)
        B.nm_heff(mesh, m, h, B.NM_T_ALL, 0.0)
        torch.cuda.synchronize()
        assert not torch.any(h)
        with pytest.raises(B.NMError):
            B.nm_llg_step(mesh, m, B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0), B.NM_RK4, B.NM_T_ALL, t_end=1e-13)
    finally:
        B.nm_mesh_destroy(mesh)
