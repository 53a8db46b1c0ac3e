"""Optional allocator hooks of nm_mesh_desc (the boundary's nm_allocator):
a mesh whose device memory comes from torch's caching allocator runs the
same kernels with the same results, torch counts its memory while it lives
and gets it back when it is destroyed, and an allocator that refuses makes
nm_mesh_create fail with NM_ENOMEM."""
import ctypes

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


def _run(p, allocator=None):
    mesh = B.mesh_from_problem(p, allocator=allocator)
    try:
        held = torch.cuda.memory_allocated()
        m = torch.as_tensor(p["m0"], device="cuda").contiguous()
        clk = B.nm_clock(0.0, 1e-14, 0, 0, 0, 0.0)
        B.nm_llg_step(mesh, m, clk, B.NM_DP45, B.NM_T_ALL, t_end=2e-12)
        torch.cuda.synchronize()
        return m, held, (clk.accepted, clk.rejected)
    finally:
        B.nm_mesh_destroy(mesh)


def test_torch_owns_the_mesh_memory_and_results_are_unchanged():
    p = synth.small_random((20, 12, 4), (2e-9, 2.5e-9, 3e-9), seed=91)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    alloc = B.TorchAllocator()
    m1, held, log1 = _run(p, alloc)
    fp = B.nm_mesh_footprint_bytes(p["n"], p["h"])
    # the mesh's buffers (most of its footprint) sat in torch's pool
    assert held - base >= 0.5 * fp, (held - base, fp)
    assert not alloc.live   # everything given back at destroy
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base <= m1.numel() * 4 + 4096
    m2, _, log2 = _run(p)
    assert torch.equal(m1, m2) and log1 == log2


class _Refusing:
    def __init__(self):
        self.calls = 0

        def _alloc(nbytes, ctx):
            self.calls += 1
            return None

        def _free(ptr, ctx):
            pass

        self._c = B.nm_allocator(B.ALLOC_FN(_alloc), B.FREE_FN(_free), None)

    def hooks(self):
        return self._c


def test_refusing_allocator_fails_cleanly():
    p = synth.small_random((8, 6, 2), (2e-9,) * 3, seed=92)
    a = _Refusing()
    with pytest.raises(B.NMError) as ei:
        B.mesh_from_problem(p, allocator=a, tensor=False)
    assert ei.value.status == B.NM_ENOMEM and a.calls >= 1
