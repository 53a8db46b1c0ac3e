"""Solve server (continuous batching) on the GPU: each result is the same alone,
in the mix and through nm_llg_step (the single-mesh kernels), served solves
match the float64 oracle node by node, admission respects the memory budget,
request semantics, and the batched server beats the one-at-a-time loop."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from helpers import to_oracle
from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import synth

pytestmark = pytest.mark.gpu

T_END = 4e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def _nn(p):
    n1, n2, n3 = p["n"]
    return (n1 + 1) * (n2 + 1) * (n3 + 1)


def _serve(reqs, max_active, budget=0, t_end=T_END):
    srv = B.nm_server_create(max_active=max_active, n_streams=4, attempts_per_launch=8, hbm_budget=budget)
    try:
        tickets = [B.nm_serve_submit(srv, p, t_end=t_end) for p in reqs]
        outs, results = [], []
        for tk, p in zip(tickets, reqs):
            m = np.empty(3 * _nn(p), dtype=np.float32)
            r = B.nm_serve_poll(srv, tk, timeout_ms=120000, m_out=m)
            assert r is not None and r.status == B.NM_OK
            outs.append(m)
            results.append(r)
    finally:
        B.nm_server_destroy(srv)
    return outs, results


def _small_stream(count, seed=7):
    return [p for _, p in synth.serving_requests(count, seed=seed, nmin=8, nmax=40, nzmax=3)]


def test_each_result_is_the_same_alone_and_in_the_mix():
    reqs = _small_stream(6)
    mix, _ = _serve(reqs, max_active=6)
    alone, _ = _serve(reqs, max_active=1)
    for a, b in zip(mix, alone):
        assert np.array_equal(a, b)


def test_each_result_is_the_single_mesh_one():
    """The batched kernels run the single-mesh kernels' code: a served solve
    (in a mix of several classes, several members per class) is bitwise the
    solve of nm_llg_step on its own mesh."""
    reqs = _small_stream(10, seed=12)
    reqs += [dict(reqs[0], m0=synth.make_problem(reqs[0]["n"], reqs[0]["h"], 8e5, 1.3e-11, 0.1, seed=50 + i)["m0"])
             for i in range(3)]
    mix, res = _serve(reqs, max_active=len(reqs))
    for p, m, r in zip(reqs, mix, res):
        mesh = B.mesh_from_problem(p)
        try:
            mt = torch.as_tensor(p["m0"], device="cuda").contiguous()
            clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
            B.nm_llg_step(mesh, mt, clk, B.NM_DP45, B.NM_T_ALL, t_end=T_END)
            single = mt.cpu().numpy().ravel()
        finally:
            B.nm_mesh_destroy(mesh)
        assert np.array_equal(m, single), p["n"]
        assert (r.accepted, r.rejected, r.rhs_evals) == (clk.accepted, clk.rejected, clk.rhs_evals)


@pytest.mark.parametrize("n", [(10, 7, 2), (21, 9, 1), (13, 12, 3)])
def test_served_solve_matches_the_oracle(n):
    """Served in a mix with two other requests of the same shape: every node
    against the float64 oracle's own adaptive run (few steps from a random
    start, so the step sequences agree)."""
    ps = [synth.make_problem(n, (3e-9,) * 3, 8e5, 1.3e-11, 0.1, seed=3 + i) for i in range(3)]
    ms, rs = _serve(ps, max_active=3, t_end=T_END)
    for p, m, r in zip(ps, ms, rs):
        om, omat, m0 = to_oracle(p)
        want, log = oracle.dp45_solve(om, omat, m0, 0.0, T_END, 1e-14, rtol=1e-5, atol=1e-5)
        g = m.reshape(want.shape).astype(np.float64)
        assert abs(r.t - T_END) < 1e-24
        assert r.accepted == sum(1 for x in log if x[2])
        assert np.abs(g - want).max() <= 1e-4


def test_served_long_films_are_the_single_mesh_ones():
    """Films with 512- and 1024-point y columns, two members per class so
    the batched film convolution runs: each served result is bitwise
    nm_llg_step's on its own mesh."""
    reqs = [synth.make_problem(n, (3e-9, 3e-9, 3e-9), 8e5, 1.3e-11, 0.1, seed=90 + i)
            for i, n in enumerate([(6, 140, 1), (6, 140, 1), (9, 300, 1), (9, 300, 1)])]
    mix, res = _serve(reqs, max_active=len(reqs))
    for p, m, r in zip(reqs, mix, res):
        mesh = B.mesh_from_problem(p)
        try:
            mt = torch.as_tensor(p["m0"], device="cuda").contiguous()
            clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
            B.nm_llg_step(mesh, mt, clk, B.NM_DP45, B.NM_T_ALL, t_end=T_END)
            single = mt.cpu().numpy().ravel()
        finally:
            B.nm_mesh_destroy(mesh)
        assert np.array_equal(m, single), p["n"]
        assert (r.accepted, r.rejected, r.rhs_evals) == (clk.accepted, clk.rejected, clk.rhs_evals)


def _material_requests():
    """Requests carrying every optional cell array the server takes:
    uniaxial Ku and easy axes, a per-cell field, DMI of both kinds, cubic
    anisotropy (two members of each class, so the classes batch)."""
    out = []
    for i, (dmi, kind, cubic) in enumerate([(True, "interfacial", False), (True, "interfacial", False),
                                            (True, "bulk", True), (True, "bulk", True),
                                            (False, "interfacial", True), (False, "interfacial", False)]):
        p = synth.small_random((12, 9, 3), (2e-9, 2.5e-9, 3e-9), seed=80 + i, dmi=dmi, dmi_type=kind,
                               cubic=cubic, ku_range=(-2e5, 5e5))
        out.append(p)
    return out


def test_served_material_terms_are_the_single_mesh_ones():
    """A request's Ku/easy, h_cell, D (interfacial or bulk) and Kc/cubic reach
    the batched kernels: each served result is bitwise nm_llg_step's."""
    reqs = _material_requests()
    mix, res = _serve(reqs, max_active=len(reqs), t_end=2e-12)
    for p, m, r in zip(reqs, mix, res):
        mesh = B.mesh_from_problem(p)
        try:
            mt = torch.as_tensor(p["m0"], device="cuda").contiguous()
            clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
            B.nm_llg_step(mesh, mt, clk, B.NM_DP45, B.NM_T_ALL, t_end=2e-12)
            single = mt.cpu().numpy().ravel()
        finally:
            B.nm_mesh_destroy(mesh)
        assert np.array_equal(m, single)
        assert (r.accepted, r.rejected) == (clk.accepted, clk.rejected)


def test_served_material_solve_matches_the_oracle():
    """Every term at once (bulk DMI, cubic and uniaxial anisotropy, per-cell
    field): each node of the served result against the oracle's own run, to
    1 ps (6 accepted steps, the last three at the stiff modes' stability
    limit, before rounding noise there could change the step sequence)."""
    p = _material_requests()[2]
    (m,), (r,) = _serve([p], max_active=1, t_end=1e-12)
    om, omat, m0 = to_oracle(p)
    want, log = oracle.dp45_solve(om, omat, m0, 0.0, 1e-12, 1e-14, rtol=1e-5, atol=1e-5)
    assert r.accepted == sum(1 for x in log if x[2])
    assert np.abs(m.reshape(want.shape).astype(np.float64) - want).max() <= 1e-4


def test_served_request_refuses_a_drive_and_half_given_arrays():
    p = _material_requests()[0]
    srv = B.nm_server_create(max_active=1)
    try:
        q = dict(p, drive_mask=np.ones_like(p["Ms"]), drive_amp=(1e3, 0.0, 0.0))
        with pytest.raises(ValueError):
            B.nm_serve_submit(srv, q)
        with pytest.raises(B.NMError) as ei:
            B.nm_serve_submit(srv, dict(p, easy=None))
        assert ei.value.status == B.NM_EINVAL
    finally:
        B.nm_server_destroy(srv)


def test_admission_respects_the_memory_budget():
    p = synth.make_problem((24, 24, 2), (3e-9,) * 3, 8e5, 1.3e-11, 0.1, seed=4)
    reqs = [dict(p, m0=synth.make_problem((24, 24, 2), (3e-9,) * 3, 8e5, 1.3e-11, 0.1, seed=10 + i)["m0"])
            for i in range(6)]
    fp = B.nm_mesh_footprint_bytes(p["n"], p["h"]) + 4 * (3 * _nn(p) + 3 * 24 * 24 * 2)
    _, res = _serve(reqs, max_active=6, budget=int(2.5 * fp))
    events = sorted([(r.t_admit, 1) for r in res] + [(r.t_done, -1) for r in res])
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 2


def test_request_that_never_fits_is_refused():
    p = _small_stream(1)[0]
    srv = B.nm_server_create(max_active=4, hbm_budget=1024)
    try:
        tk = B.nm_serve_submit(srv, p, t_end=T_END)
        r = B.nm_serve_poll(srv, tk, timeout_ms=60000)
        assert r is not None and r.status == B.NM_EBUDGET and r.accepted == 0
    finally:
        B.nm_server_destroy(srv)


def test_poll_semantics():
    srv = B.nm_server_create(max_active=2)
    try:
        with pytest.raises(B.NMError) as ei:
            B.nm_serve_poll(srv, 12345)
        assert ei.value.status == B.NM_EINVAL
        p = _small_stream(1, seed=9)[0]
        tk = B.nm_serve_submit(srv, p, t_end=T_END)
        r = None
        t0 = time.time()
        while r is None and time.time() - t0 < 120:
            r = B.nm_serve_poll(srv, tk, timeout_ms=50)
        assert r is not None and r.status == B.NM_OK and r.accepted > 0
        assert r.t_submit <= r.t_admit <= r.t_done
        with pytest.raises(B.NMError):
            B.nm_serve_poll(srv, tk)   # a polled ticket is forgotten
    finally:
        B.nm_server_destroy(srv)


def test_batched_server_beats_the_plain_loop():
    """16 small solves long enough (20 ps) that stepping, not set-up, dominates."""
    reqs = _small_stream(16, seed=11)
    _serve(reqs[:2], max_active=2, t_end=1e-12)   # warm-up: tuner caches, code objects
    t0 = time.perf_counter()
    _serve(reqs, max_active=16, t_end=2e-11)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    _serve(reqs, max_active=1, t_end=2e-11)
    t_plain = time.perf_counter() - t0
    print("16 solves: batched %.3f s, one at a time %.3f s" % (t_batch, t_plain), flush=True)
    assert t_batch < t_plain
