"""The allocation-free tensor set-up (nm_demag_tensor_init_noalloc, through
the C ABI) against nm_demag_tensor_init: the demag field of meshes set up
either way is bitwise the same, for two calls in a row with a smaller mesh
second (the static scratch keeps the first call's contents), and a grid whose
set-up needs more scratch than the entry point has is refused."""
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


def _demag(p, noalloc):
    mesh = B.mesh_from_problem(p, tensor=False)
    try:
        if noalloc:
            B.nm_demag_tensor_init_noalloc(mesh)
        else:
            B.nm_demag_tensor_init(mesh)
        # the same FFT tile widths on both meshes (the widest)
        B.nm_mesh_tuning(mesh, y=0, z=0)
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        h = torch.empty_like(m)
        B.nm_heff(mesh, m, h, B.NM_T_DEMAG, 0.0)
        hc = torch.empty((3,) + tuple(reversed(p["n"])), device="cuda")
        B.nm_demag_cell_field(mesh, m, hc)
        torch.cuda.synchronize()
        return h.cpu().numpy(), hc.cpu().numpy()
    finally:
        B.nm_mesh_destroy(mesh)


def test_noalloc_tensor_matches_the_allocating_one_twice_in_a_row():
    big = synth.small_random((40, 24, 6), (2e-9, 2.5e-9, 3e-9), seed=31)
    small = synth.small_random((9, 5, 2), (3e-9, 2e-9, 2e-9), seed=32)
    film = synth.small_random((33, 17, 1), (4e-9, 4e-9, 5e-9), seed=33)
    for p in (big, small, film):
        want_h, want_c = _demag(p, noalloc=False)
        got_h, got_c = _demag(p, noalloc=True)
        assert np.isfinite(want_h).all() and np.abs(want_h).max() > 0
        assert np.array_equal(got_h, want_h)
        assert np.array_equal(got_c, want_c)


def test_noalloc_refuses_grids_beyond_its_scratch():
    # 256 x 256 x 64 cells: about 660 MB of float64 temporaries
    n = (256, 256, 64)
    p = synth.make_problem(n, (2e-9,) * 3, 8e5, 1.3e-11, 0.1, m0=(1.0, 0.0, 0.0))
    mesh = B.mesh_from_problem(p, tensor=False)
    try:
        with pytest.raises(B.NMError) as ei:
            B.nm_demag_tensor_init_noalloc(mesh)
        assert ei.value.status == B.NM_EINVAL
        assert "scratch" in str(ei.value)
        # the mesh is still usable through the allocating set-up
        B.nm_demag_tensor_init(mesh)
    finally:
        B.nm_mesh_destroy(mesh)
