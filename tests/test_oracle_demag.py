"""Pins of the oracle's demagnetisation tensor and FFT convolution (Sec. 3.2)."""
import numpy as np
import pytest

import oracle
from oracle.newell import GL_BANDS, NEWELL_RADIUS, newell_far, newell_near

from helpers import aharoni_factor, rel_l2, to_oracle
from paper_2411_11725_amd import synth


def test_cube_self_term_is_one_third():
    for hh in (1.0, 2e-9):
        N0 = oracle.newell_offset(([0], [0], [0]), (hh, hh, hh))[:, 0]
        assert np.allclose(N0[:3], 1.0 / 3.0, rtol=0, atol=1e-14)
        assert np.allclose(N0[3:], 0.0, atol=1e-15)


def test_self_term_trace_is_one_for_prisms():
    rng = np.random.default_rng(1)
    for _ in range(10):
        h = tuple(rng.uniform(0.2, 5.0, 3))
        N0 = oracle.newell_offset(([0], [0], [0]), h)[:, 0]
        assert abs(N0[:3].sum() - 1.0) < 1e-13
        assert np.all(N0[:3] > 0)
        # the flattest edge gets the largest factor
        assert np.argmax(N0[:3]) == int(np.argmin(h))


def test_trace_vanishes_off_the_self_term():
    """Away from the source cell the field is harmonic: tr N(d) = 0."""
    h = (2e-9, 2.5e-9, 3e-9)
    d = np.array([(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1), (3, 2, 0), (2, 5, 1),
                  (7, 1, 3), (12, 9, 4), (40, 3, 2), (90, 70, 7)]).T
    N = oracle.newell_offset(d, h)
    scale = np.abs(N).max(axis=0)
    assert np.all(np.abs(N[:3].sum(axis=0)) <= 1e-9 * scale)


def test_parities_and_axis_permutation():
    h = (1.0, 1.4, 0.8)
    d = np.array([(1, 2, 3), (4, 1, 2), (6, 5, 1), (2, 0, 7)]).T
    N = oracle.newell_offset(d, h)
    for s in [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]:
        Ns = oracle.newell_offset(d * np.array(s)[:, None], h)
        sx, sy, sz = s
        want = N * np.array([1, 1, 1, sx * sy, sx * sz, sy * sz])[:, None]
        # Newell cancellation amplifies the rounding of X + e h differently
        # for mirrored offsets: compare at 1e-11 of each offset's scale
        assert np.all(np.abs(Ns - want) <= 1e-11 * np.abs(N).max(axis=0))
    # swapping the x and y axes of the grid swaps the components accordingly
    hp = (h[1], h[0], h[2])
    dp = d[[1, 0, 2]]
    Np = oracle.newell_offset(dp, hp)
    assert np.all(np.abs(Np[[1, 0, 2, 3, 5, 4]] - N) <= 1e-11 * np.abs(N).max(axis=0))


def test_far_field_approaches_point_dipole():
    """N(d) -> V N_dip(X) with a relative error that falls as (h/r)^2."""
    h = (2.0, 1.0, 1.5)
    V = h[0] * h[1] * h[2]
    errs = []
    for s in (8, 16, 32, 64):
        d = np.array([[s], [s // 2], [s // 4]])
        N = oracle.newell_offset(d, h)[:, 0]
        X = d[:, 0] * np.array(h)
        dip = V * oracle.dipole_tensor(*X)
        errs.append(np.abs(N - dip).max() / np.abs(dip).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 3.5) & (ratios < 4.5)), ratios


def test_newell_and_quadrature_agree_at_the_switch():
    """The two routes for N(d) agree to ~1e-10 where the oracle switches."""
    for h in [(1.0, 1.0, 1.0), (1.0, 1.0, 3 / 3.9), (0.8, 0.8, 1.0)]:
        hs = max(h)
        hh = tuple(v / hs for v in h)
        for d in [(4, 1, 0), (3, 2, 1), (4, 2, 1), (5, 0, 0), (2, 3, 2)]:
            X = np.array(d, dtype=float) * np.array(hh)
            near = newell_near(X[0], X[1], X[2], hh)
            far = newell_far(X[0], X[1], X[2], hh, GL_BANDS[0][1])
            assert np.abs(near - far).max() <= 2e-10 * np.abs(near).max()


def test_quadrature_converged_in_every_band():
    h = (1.0, 1.0, 0.77)
    lo = NEWELL_RADIUS
    for hi, npts in GL_BANDS:
        r = lo * 1.0001
        X = np.array([r, 0.0, 0.0])
        a = newell_far(*X, h, npts)
        b = newell_far(*X, h, npts + 4)
        assert np.abs(a - b).max() <= 2e-11 * np.abs(b).max()
        lo = hi if np.isfinite(hi) else lo


def _uniform_problem(n, h, mdir):
    mesh = oracle.Mesh(n, h)
    cs = mesh.cell_shape
    Ms = 8e5
    mat = oracle.Material(Ms=np.full(cs, Ms), A=np.zeros(cs), alpha=np.zeros(cs))
    m = np.broadcast_to(np.asarray(mdir, float).reshape(3, 1, 1, 1), (3,) + mesh.node_shape).copy()
    return mesh, mat, m, Ms


def test_uniform_cube_mean_field_is_minus_m_over_three():
    for nn in (1, 3, 4):
        mesh, mat, m, Ms = _uniform_problem((nn, nn, nn), (2e-9,) * 3, (1.0, 0.0, 0.0))
        H = oracle.demag_cell_field(mesh, mat, m)
        assert abs(H[0].mean() / Ms + 1.0 / 3.0) < 1e-12
        assert abs(H[1].mean()) < 1e-12 * Ms and abs(H[2].mean()) < 1e-12 * Ms


def test_box_mean_tensor_has_unit_trace():
    n, h = (6, 3, 2), (2e-9, 3e-9, 1.5e-9)
    tr = 0.0
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1.0
        mesh, mat, m, Ms = _uniform_problem(n, h, e)
        tr += -oracle.demag_cell_field(mesh, mat, m)[j].mean() / Ms
    assert abs(tr - 1.0) < 1e-12


@pytest.mark.parametrize("n,h", [((6, 5, 3), (2e-9, 3e-9, 2.5e-9)),
                                 ((9, 4, 1), (3.9e-9, 3.9e-9, 3e-9)),
                                 ((4, 4, 4), (2e-9, 2e-9, 2e-9))])
def test_fft_convolution_equals_direct_sum(n, h):
    p = synth.small_random(n, h, seed=21)
    mesh, mat, m = to_oracle(p)
    Hf = oracle.demag_cell_field(mesh, mat, m)
    Hd = oracle.demag_cell_field_direct(mesh, mat, m)
    assert rel_l2(Hf, Hd) < 1e-12


def test_result_does_not_depend_on_padding():
    p = synth.small_random((5, 6, 3), (2e-9, 2e-9, 3e-9), seed=22)
    mesh, mat, m = to_oracle(p)
    H1 = oracle.demag_cell_field(mesh, mat, m, pad=(10, 12, 6))
    H2 = oracle.demag_cell_field(mesh, mat, m, pad=(9, 16, 7))
    H3 = oracle.demag_cell_field(mesh, mat, m, pad=(16, 11, 5))
    assert rel_l2(H1, H2) < 1e-12 and rel_l2(H1, H3) < 1e-12


def test_single_layer_tensor_has_no_z_coupling():
    """For N3 = 1 only z-offset 0 occurs and N_xz = N_yz = 0 there."""
    N = oracle.newell_octant((6, 5, 1), (3.9e-9, 3.9e-9, 3e-9))
    assert np.abs(N[4:]).max() <= 1e-15 * np.abs(N).max()


def test_fft_tensor_spectrum_is_real():
    from oracle.field import padded_tensor
    n = (6, 5, 4)
    oc = oracle.newell_octant(n, (2e-9, 2.5e-9, 3e-9))
    Nk = np.fft.fftn(padded_tensor(oc, n, (12, 10, 8)), axes=(1, 2, 3))
    assert np.abs(Nk.imag).max() <= 1e-12 * np.abs(Nk.real).max()


@pytest.mark.parametrize("n,h", [((6, 4, 3), (2e-9, 2.5e-9, 3e-9)), ((12, 5, 1), (3e-9, 2e-9, 1.5e-9)),
                                 ((3, 3, 9), (2e-9, 2e-9, 2e-9))])
def test_box_mean_field_matchesaharoni_factor(n, h):
    """A uniformly magnetised box of cells: the mean cell field along each
    axis is -N M with N the prism's closed-form demagnetising factor (the
    cell-averaged tensor sums to the body-averaged one exactly), through the
    Newell near field, the quadrature far field and the FFT convolution."""
    mesh = oracle.Mesh(n, h)
    cs = mesh.cell_shape
    mat = oracle.Material(Ms=np.full(cs, 1e6), A=np.zeros(cs), alpha=np.zeros(cs))
    half = [n[i] * h[i] / 2 for i in range(3)]
    assert aharoni_factor(1.0, 1.0, 1.0) == pytest.approx(1 / 3, rel=1e-14)
    for axis in range(3):
        m = np.zeros((3,) + mesh.node_shape)
        m[axis] = 1.0
        H = oracle.demag_cell_field(mesh, mat, m)
        others = [half[(axis + 1) % 3], half[(axis + 2) % 3]]
        want = aharoni_factor(others[0], others[1], half[axis])
        assert abs(-H[axis].mean() / 1e6 - want) <= 1e-11
