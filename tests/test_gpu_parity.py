"""GPU (HIP, float32) vs the float64 oracle, element by element, through the C ABI.

Tolerances: the relative L2 field error per evaluation is held to 1e-5 (the
stated bound for every evaluation of the effective field); the float64
tensor set-up is held to the accuracy of its quadrature (~1e-12 of the
largest entry); trajectories to max |dm| <= 1e-4 after the stated steps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle.field import ALL_TERMS, ANISOTROPY, DEMAG, EXCHANGE, ZEEMAN
from helpers import aharoni_factor, gpu_replay_steps, rel_l2, to_oracle
from paper_2411_11725_amd import binding as B
from paper_2411_11725_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()  # a missing library is an error, not a skip


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _field(p, terms, t=0.0, kind="heff"):
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        out = torch.empty_like(m)
        if kind == "heff":
            B.nm_heff(mesh, m, out, terms, t)
        else:
            B.nm_llg_rhs(mesh, m, out, terms, t)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)


SHAPES = [
    ((5, 3, 2), (2e-9, 3e-9, 2.5e-9)),
    ((13, 7, 3), (2e-9, 2e-9, 2e-9)),
    ((16, 16, 4), (2e-9, 2e-9, 2e-9)),
    ((9, 4, 1), (3.9e-9, 3.9e-9, 3e-9)),
    ((33, 17, 1), (4e-9, 4e-9, 5e-9)),
    ((20, 12, 5), (3e-9, 2e-9, 4e-9)),
    ((2, 2, 1), (2e-9, 2e-9, 2e-9)),
]


@pytest.mark.parametrize("n,h", [((16, 16, 4), (2e-9,) * 3), ((24, 10, 1), (3.9e-9, 3.9e-9, 3e-9)),
                                 ((12, 9, 7), (4e-9, 4e-9, 5e-9)), ((40, 3, 2), (1e-9, 2e-9, 3e-9))])
def test_newell_octant_matches_oracle(n, h):
    out = torch.empty((6,) + (n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    B.nm_newell_octant(n, h, out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    o = oracle.newell_octant(n, h)
    scale = np.abs(o).max()
    local = np.abs(o).max(axis=0, keepdims=True)
    assert np.abs(g - o).max() <= 1e-12 * scale
    assert np.all(np.abs(g - o) <= 1e-9 * local + 1e-15 * scale)


@pytest.mark.parametrize("n,h", SHAPES)
def test_demag_cell_field_matches_oracle(n, h):
    p = synth.small_random(n, h, seed=41)
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        out = torch.empty((3,) + (n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
        B.nm_demag_cell_field(mesh, m, out)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
    finally:
        B.nm_mesh_destroy(mesh)
    om, omat, om0 = to_oracle(p)
    want = oracle.demag_cell_field(om, omat, om0)
    assert rel_l2(g, want) <= 1e-5


@pytest.mark.parametrize("n,h", SHAPES)
@pytest.mark.parametrize("terms", [EXCHANGE, DEMAG, ANISOTROPY, ZEEMAN, ALL_TERMS])
def test_heff_matches_oracle(n, h, terms):
    p = synth.small_random(n, h, seed=43)
    g = _field(p, terms)
    om, omat, om0 = to_oracle(p)
    want = oracle.heff(om, omat, om0, terms)
    assert rel_l2(g, want) <= 1e-5


@pytest.mark.parametrize("n,h", SHAPES[:3] + SHAPES[4:5])
def test_anisotropy_of_either_sign_matches_oracle(n, h):
    """Easy-axis (Ku > 0) and easy-plane (Ku < 0) cells mixed in one mesh."""
    p = synth.small_random(n, h, seed=48, ku_range=(-5e5, 5e5))
    assert (p["Ku"] < 0).any() and (p["Ku"] > 0).any()
    om, omat, om0 = to_oracle(p)
    for terms in (ANISOTROPY, ALL_TERMS):
        g = _field(p, terms)
        assert rel_l2(g, oracle.heff(om, omat, om0, terms)) <= 1e-5


@pytest.mark.parametrize("n,h", SHAPES[:4])
def test_llg_rhs_matches_oracle(n, h):
    p = synth.small_random(n, h, seed=44)
    g = _field(p, ALL_TERMS, kind="rhs")
    om, omat, om0 = to_oracle(p)
    want = oracle.llg_rhs(om, omat, om0)
    assert rel_l2(g, want) <= 1e-5


def test_drive_field_follows_time():
    p = synth.magnonic(n=(24, 8, 1))
    for t in (0.0, 0.013e-9, 0.07e-9):
        g = _field(p, ZEEMAN, t=t)
        om, omat, om0 = to_oracle(p)
        assert rel_l2(g, oracle.heff(om, omat, om0, ZEEMAN, t)) <= 1e-6


@pytest.mark.parametrize("n,h", SHAPES[:5])
def test_energies_match_oracle(n, h):
    p = synth.small_random(n, h, seed=45)
    mesh = B.mesh_from_problem(p)
    try:
        e = B.nm_energy(mesh, _dev(p["m0"]), B.NM_T_ALL, 0.0)
    finally:
        B.nm_mesh_destroy(mesh)
    om, omat, om0 = to_oracle(p)
    want = oracle.energies(om, omat, om0)
    for k in ("exchange", "demag", "anisotropy", "zeeman", "total"):
        assert abs(e[k] - want[k]) <= 1e-5 * abs(want[k]) + 1e-30, k


def test_padded_lengths_up_to_1024():
    """Longest transforms: P1 = 1024 (x through a 512-point complex FFT),
    P2 = 1024 and P3 = 1024."""
    for n in [(300, 3, 1), (5, 300, 2), (3, 2, 260)]:
        p = synth.small_random(n, (2e-9, 2e-9, 2e-9), seed=46, anis=False, field=False)
        g = _field(p, DEMAG)
        om, omat, om0 = to_oracle(p)
        assert rel_l2(g, oracle.heff(om, omat, om0, DEMAG)) <= 1e-5, n


@pytest.mark.parametrize("n", [(5, 300, 1), (9, 200, 1), (40, 100, 1), (3, 129, 1), (70, 128, 1)])
def test_film_long_columns_match_oracle(n):
    """Single-layer films with the film convolution's long y columns (padded
    lengths 256, 512, 1024: four, two and one column per block), ragged kx
    column counts, and data rows up to exactly half the padded length (128
    of 256)."""
    p = synth.small_random(n, (3e-9, 2.5e-9, 3e-9), seed=47, anis=False, field=False)
    g = _field(p, DEMAG)
    om, omat, om0 = to_oracle(p)
    want = oracle.heff(om, omat, om0, DEMAG)
    assert rel_l2(g, want) <= 1e-5, n
    assert np.abs(g - want).max() <= 1e-4 * np.abs(want).max(), n


@pytest.mark.parametrize("n", [(512, 3, 1), (3, 512, 2), (2, 3, 512), (512, 2, 2)])
def test_largest_axis_length_matches_oracle(n):
    """512 cells on an axis, the most a mesh takes (padded to 1024, the data
    filling exactly half of the transform)."""
    p = synth.small_random(n, (2e-9, 2e-9, 2e-9), seed=48, anis=False, field=False)
    g = _field(p, DEMAG)
    om, omat, om0 = to_oracle(p)
    want = oracle.heff(om, omat, om0, DEMAG)
    assert rel_l2(g, want) <= 1e-5, n
    assert np.abs(g - want).max() <= 1e-4 * np.abs(want).max(), n


def test_results_are_bitwise_reproducible():
    p = synth.small_random((13, 7, 3), (2e-9,) * 3, seed=47)
    a = _field(p, ALL_TERMS)
    b = _field(p, ALL_TERMS)
    assert np.array_equal(a, b)


def test_rk4_standard_cube_trajectory():
    """16 x 16 x 4 cells, random start, RK4 dt = 1e-14 s for 1000 steps."""
    p = synth.standard_cube()
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_RK4, B.NM_T_ALL, t_end=1000 * 1e-14)
        g = m.cpu().numpy().astype(np.float64)
        e_gpu = B.nm_energy(mesh, m, B.NM_T_ALL)
    finally:
        B.nm_mesh_destroy(mesh)
    assert clk.accepted == 1000 and clk.rhs_evals == 4000
    assert abs(clk.t - 1e-11) < 1e-25
    om, omat, om0 = to_oracle(p)
    want, _ = oracle.rk4_solve(om, omat, om0, 1e-14, 1000)
    assert np.abs(g - want).max() <= 1e-4
    e_or = oracle.energies(om, omat, want)
    assert abs(e_gpu["total"] - e_or["total"]) <= 1e-4 * abs(e_or["total"])


@pytest.mark.parametrize("n", [(40, 24, 6), (130, 20, 3)])
def test_every_tile_width_gives_the_same_field(n):
    """The tuner's block widths of the y passes and the z convolution compute
    each column identically: the field is bitwise the same for every width."""
    p = synth.small_random(n, (2e-9, 2e-9, 3e-9), seed=50)
    mesh = B.mesh_from_problem(p)
    try:
        chosen = B.nm_mesh_tuning(mesh)
        assert all(0 <= w <= 2 for w in chosen)
        m = _dev(p["m0"])
        outs = []
        for w in range(3):
            assert B.nm_mesh_tuning(mesh, y=w, z=w) == (w, w)
            h = torch.empty_like(m)
            B.nm_heff(mesh, m, h, ALL_TERMS, 0.0)
            torch.cuda.synchronize()
            outs.append(h.cpu().numpy())
        with pytest.raises(B.NMError):
            B.nm_mesh_tuning(mesh, y=3)
    finally:
        B.nm_mesh_destroy(mesh)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    om, omat, om0 = to_oracle(p)
    assert rel_l2(outs[0], oracle.heff(om, omat, om0, ALL_TERMS)) <= 1e-5


@pytest.mark.parametrize("n1", [20, 83, 84, 100, 168, 169, 200, 296, 297, 350, 424, 425, 450])
def test_long_rows_match_oracle(n1):
    """Rows from 21 to 451 nodes: every LDS window size of the node kernel
    (5, 7, 10 and 13 items per thread) on both sides of each switch (rows of
    84/85, 169/170, 297/298 and 425/426 nodes), its direct-load form for rows
    too long for a window, and the x passes up to 512-point half rows."""
    p = synth.small_random((n1, 5, 3), (2e-9, 3e-9, 2.5e-9), seed=51, ku_range=(-5e5, 5e5))
    om, omat, om0 = to_oracle(p)
    g = _field(p, ALL_TERMS)
    assert rel_l2(g, oracle.heff(om, omat, om0, ALL_TERMS)) <= 1e-5
    r = _field(p, ALL_TERMS, kind="rhs")
    assert rel_l2(r, oracle.llg_rhs(om, omat, om0)) <= 1e-5


def test_rk4_calls_queue_without_waiting_and_keep_the_clock():
    """RK4 calls return once queued: successive calls (a max_steps stop, then a
    shortened last step landing on t_end, then single steps with a drive in
    time) give the oracle's states and the exact clock."""
    p = synth.small_random((9, 7, 3), (2e-9, 2.5e-9, 3e-9), seed=49)
    p["drive_mask"] = np.ones((3, 7, 9), dtype=np.float32)
    p["drive_amp"] = (0.0, 2e4, 0.0)
    p["drive_freq"] = 2e10
    mesh = B.mesh_from_problem(p)
    om, omat, om0 = to_oracle(p)
    dt, t_end = 3e-15, 3e-15 * 7.4
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, dt, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_RK4, B.NM_T_ALL, t_end=t_end, max_steps=3)
        assert clk.accepted == 3 and abs(clk.t - 3 * dt) < 1e-28
        B.nm_llg_step(mesh, m, clk, B.NM_RK4, B.NM_T_ALL, t_end=t_end)
        assert clk.accepted == 8 and clk.t == t_end and clk.rhs_evals == 32
        for _ in range(3):
            B.nm_llg_step(mesh, m, clk, B.NM_RK4, B.NM_T_ALL, t_end=clk.t + dt, max_steps=1)
        g = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    want, t = om0, 0.0
    for k in range(8):
        h = min(dt, t_end - t)
        want = oracle.rk4_step(om, omat, want, t, h)
        t = t_end if k == 7 else t + h
    for _ in range(3):
        want = oracle.rk4_step(om, omat, want, t, dt)
        t += dt
    assert abs(clk.t - t) < 1e-27 and clk.accepted == 11
    assert np.abs(g - want).max() <= 1e-5


def _film_problem():
    return synth.make_problem((32, 16, 1), (3.9e-9, 3.9e-9, 3e-9), 8e5, 1.3e-11, 0.02,
                              m0=(np.cos(0.17), np.sin(0.17), 0.0),
                              h_uniform=(-25e-3 / synth.MU0_SI, 4e-3 / synth.MU0_SI, 0.0))


def _film_dp45(max_steps, t_end=0.05e-9, dt0=1e-14):
    p = _film_problem()
    mesh = B.mesh_from_problem(p)
    log = torch.zeros(3 * 4000, dtype=torch.float64, device="cuda")
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, dt0, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=t_end, rtol=1e-5, atol=1e-5,
                      log=log, max_steps=max_steps)
        g = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    L = log.cpu().numpy().reshape(-1, 3)[: clk.accepted + clk.rejected]
    assert sum(1 for x in L if x[2] > 0.5) == clk.accepted
    return p, g, [(t, dt, ok > 0.5) for t, dt, ok in L], clk


def _replay(p, steps):
    """The GPU state after taking the given accepted steps (t, dt)."""
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        gpu_replay_steps(B, mesh, m, steps, B.NM_T_ALL)
        return m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)


def test_dp45_split_calls_follow_the_same_steps():
    """The same adaptive run as one call and as calls of 3, 1, 5, 2, ... steps
    (every last replay of a call is a smaller graph): the same accepted steps
    and the same state, up to the rounding of the first stage recomputed at
    each call."""
    p, g1, log1, clk1 = _film_dp45(max_steps=1 << 40, t_end=0.01e-9)
    mesh = B.mesh_from_problem(p)
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        sizes = [3, 1, 5, 2, 7, 4, 6]
        k = 0
        while clk.t < 0.01e-9:
            before = clk.accepted
            B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=0.01e-9, rtol=1e-5, atol=1e-5,
                          max_steps=sizes[k % len(sizes)])
            assert clk.accepted - before <= sizes[k % len(sizes)]
            k += 1
        g2 = m.cpu().numpy().astype(np.float64)
    finally:
        B.nm_mesh_destroy(mesh)
    assert k >= 3 and clk.t == 0.01e-9
    assert clk.accepted == clk1.accepted
    assert np.abs(g2 - g1).max() <= 1e-5


def test_dp45_controller_log_matches_oracle():
    """The GPU controller's attempt log (t, dt, accepted) against the float64
    oracle's own adaptive run from a step far too large: two rejections, the
    no-growth step after them, then error-driven steps; the same accept /
    reject pattern, and t and dt to the accuracy of the float32 error
    estimate (a cancelling combination of the stage derivatives whose
    rounding reaches ~1e-5 of the norm, a fifth of that in the step; 2.5e-6
    measured).  The comparison covers the first 6 attempts: at the steps
    that follow (~1.87e-12 s) the film's stiff exchange modes lie outside
    the Dormand-Prince stability region, and their rounding noise grows ~8x
    per step until the error estimate sees it, after 2-3 more steps in
    float32 and ~10 more in float64 (the oracle's own run is rejected there),
    so the two logs part by construction, not by a fault of either."""
    n_att = 6
    p, _, log, clk = _film_dp45(max_steps=1 << 40, t_end=0.05e-9, dt0=2e-11)
    om, omat, om0 = to_oracle(p)
    _, olog = oracle.dp45_solve(om, omat, om0, 0.0, 0.05e-9, 2e-11, rtol=1e-5, atol=1e-5, max_attempts=n_att)
    assert len(log) >= n_att and len(olog) == n_att
    assert [x[2] for x in olog] == [False, False, True, True, True, True]
    assert [bool(x[2]) for x in log[:n_att]] == [x[2] for x in olog]
    # the no-growth rule: the step after the accepted retry keeps its size
    assert log[3][1] == log[2][1]
    worst = max(max(abs(a[0] - b[0]) / max(b[0], b[1]), abs(a[1] - b[1]) / b[1])
                for a, b in zip(log[:n_att], olog))
    assert worst <= 2e-5, worst


def test_dp45_replay_first_steps_pointwise():
    """Replay parity, node by node: the GPU takes the oracle's first accepted
    steps (inside the stability region of the exchange modes)."""
    p = _film_problem()
    om, omat, om0 = to_oracle(p)
    want, olog = oracle.dp45_solve(om, omat, om0, 0.0, 0.05e-9, 1e-14, rtol=1e-5, atol=1e-5, max_accepted=5)
    steps = [(t, dt) for t, dt, ok in olog if ok]
    assert len(steps) == 5
    g = _replay(p, steps)
    assert np.abs(g - want).max() <= 1e-6


def test_dp45_film_replay_and_independent_parity():
    """Full adaptive run with a field step.  Replay mode: the GPU takes the
    accepted steps of the oracle's run with steps capped at 4e-13 s, inside
    the stability region of the film's exchange modes (uncapped, the
    controller first takes steps outside it, where float32 rounding noise
    grows ~8x per step), compared node by node and through the film average.
    Independent mode: the GPU's own uncapped run against the oracle's, both
    with their own controllers; the film average agrees at the tolerance
    scale."""
    p = _film_problem()
    om, omat, om0 = to_oracle(p)
    want, olog = oracle.dp45_solve(om, omat, om0, 0.0, 0.05e-9, 1e-14, rtol=1e-5, atol=1e-5, dt_max=4e-13)
    steps = [(t, dt) for t, dt, ok in olog if ok]
    assert len(steps) > 100
    g = _replay(p, steps)
    mean = lambda a: a.mean(axis=(1, 2, 3))
    free, _ = oracle.dp45_solve(om, omat, om0, 0.0, 0.05e-9, 1e-14, rtol=1e-5, atol=1e-5)
    _, gi, _, clk = _film_dp45(max_steps=1 << 40)
    print("replay of %d capped steps: <m> %.2e, nodes %.2e; independent <m> %.2e"
          % (len(steps), np.abs(mean(g) - mean(want)).max(), np.abs(g - want).max(),
             np.abs(mean(gi) - mean(free)).max()), flush=True)
    assert np.abs(mean(g) - mean(want)).max() <= 1e-6
    assert np.abs(g - want).max() <= 1e-5
    assert abs(clk.t - 0.05e-9) <= 1e-22
    assert np.abs(mean(gi) - mean(free)).max() <= 1e-4


@pytest.mark.parametrize("name", ["film", "block", "block_dmi"])
def test_full_size_workload_field(name):
    """Every node of the full-size workloads (256x64x1 film, 128x128x32 block,
    the block with DMI) in the launch configuration the benchmark uses."""
    p = synth.block(D=3e-3) if name == "block_dmi" else getattr(synth, name)()
    terms = ALL_TERMS
    g = _field(p, terms)
    om, omat, om0 = to_oracle(p)
    want = oracle.heff(om, omat, om0, terms)
    assert rel_l2(g, want) <= 1e-5
    f = _field(p, terms, kind="rhs")
    assert rel_l2(f, oracle.llg_rhs(om, omat, om0)) <= 1e-5


@pytest.mark.parametrize("n,h", [((128, 128, 32), (2e-9, 2e-9, 2e-9)), ((256, 64, 1), (3.9e-9, 3.9e-9, 3e-9)),
                                 ((60, 20, 45), (2e-9, 3e-9, 1.5e-9))])
def test_box_mean_field_matches_aharoni(n, h):
    """A uniformly magnetised box at the workloads' sizes: the mean cell field
    along each axis is -N M with N the prism's closed-form demagnetising
    factor (Aharoni), a property of the exact convolution at any size."""
    p = synth.make_problem(n, h, 1e6, 1e-11, 0.1, m0=(1.0, 0.0, 0.0))
    mesh = B.mesh_from_problem(p)
    half = [n[i] * h[i] / 2 for i in range(3)]
    try:
        for axis in range(3):
            m0 = np.zeros_like(p["m0"])
            m0[axis] = 1.0
            out = torch.empty((3,) + (n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
            B.nm_demag_cell_field(mesh, _dev(m0), out)
            torch.cuda.synchronize()
            got = -float(out[axis].double().mean()) / 1e6
            want = aharoni_factor(half[(axis + 1) % 3], half[(axis + 2) % 3], half[axis])
            assert abs(got - want) <= 2e-6, (axis, got, want)
    finally:
        B.nm_mesh_destroy(mesh)


@pytest.mark.parametrize("name", ["block", "film"])
def test_full_size_dp45_steps_lower_the_energy(name):
    """The benchmark's own configuration (full-size workload, DP45 graph
    replays): with static fields and alpha > 0 the total energy falls
    monotonically from call to call (dE/dt = -sum M alpha gamma' |m x H|^2)
    and |m| stays 1 to the integrator's tolerance in the RMS over nodes.  No
    renormalisation: from the block's random start the float64 oracle's own
    DP45 (rtol 1e-5) drifts by 1.2e-4 RMS and 3e-3 at the worst node of a
    16 x 16 x 8 block in 43 steps, so the worst node is not bounded here."""
    p = getattr(synth, name)()
    mesh = B.mesh_from_problem(p)
    terms = B.NM_T_ALL
    try:
        m = _dev(p["m0"])
        clk = B.nm_clock(0.0, 1e-14 if name == "block" else 1e-13, 0, 0, 0, 0.0)
        es = [B.nm_energy(mesh, m, terms, 0.0)["total"]]
        for _ in range(4):
            B.nm_llg_step(mesh, m, clk, B.NM_DP45, terms, t_end=20e-9, max_steps=10)
            es.append(B.nm_energy(mesh, m, terms, clk.t)["total"])
        norm = torch.linalg.vector_norm(m, dim=0).double()
        torch.cuda.synchronize()
        drift = float(((norm - 1) ** 2).mean().sqrt())
    finally:
        B.nm_mesh_destroy(mesh)
    assert clk.accepted == 40
    assert all(b < a for a, b in zip(es, es[1:])), es
    assert drift <= 1e-3
